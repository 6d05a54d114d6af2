/* Exercises every entry point of the oracle (oracle/oracle.c) on small matrices built here, for the
 * AddressSanitizer / UndefinedBehaviorSanitizer build of the CPU tests.  Checks a few closed-form facts
 * on the way (Dirichlet Laplacian eigenvalues) and exits non-zero on any mismatch. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int p, itmax, itmax_dacg, itmax_pcg, kmax, exit_rule;
    double tol, tol_dacg, tol_pcg, exit_xi, shift0, shift_max;
    int newton, bfgs_full, ict, lfil;
    double tau_ic;
    int jd, jd_mmin, jd_mmax;
} or_opts;

typedef struct {
    int dacg_its[32], outer_its[32], pcg_its[32], converged[32];
    double relres[32];
    long long mvp_dacg, mvp_newton;
    int bfgs_skipped, pcg_breakdowns, ntrace, status;
    double shift_used, t_factor, t_dacg, t_newton;
    int dacg_restarts;
    long long nnz_L;
    double fill;
} or_stats;

int or_solve(int n, const int *rp, const int *ci, const double *v, const or_opts *o, const double *x0, double *evals,
             double *evecs, or_stats *st, double *trace, int trace_cap);
int or_backward(int n, const int *rp, const int *ci, const double *v, int p, const double *evals,
                const double *evecs, const double *g_evals, const double *g_evecs, double tol, int itmax,
                double shift0, double shift_max, double *g_vals);
int or_tril_nnz(int n, const int *rp, const int *ci);
int or_ic0(int n, const int *rp, const int *ci, const double *v, double shift0, double shift_max, int *Lrp, int *Lci,
           double *Lv, double *shift_used);
int or_ict(int n, const int *rp, const int *ci, const double *v, int lfil, double tau, double shift0,
           double shift_max, int **Lrp, int **Lci, double **Lv, double *shift_used);
void or_free(void *p);
void or_lsolve(int n, const int *Lrp, const int *Lci, const double *Lv, const double *b, double *x);
void or_ltsolve(int n, const int *Lrp, const int *Lci, const double *Lv, const double *b, double *x);
void or_spmv(int n, const int *rp, const int *ci, const double *v, const double *x, double *y);
void or_symeig(int m, double *H, double *ev, double *Y);
void or_bfgspk_apply(int n, const int *Lrp, const int *Lci, const double *Lv, int k, const double *S,
                     const double *R, int m, const double *Q, const double *g, double *c);
int or_window_apply(int n, const int *Lrp, const int *Lci, const double *Lv, int kmax, int npush, const double *S,
                    const double *R, int m, const double *Q, const double *g, double *c);
int or_pcg_apply(int n, const int *rp, const int *ci, const double *v, const int *Lrp, const int *Lci,
                 const double *Lv, double theta, int m, const double *Q, const double *u, const double *Au,
                 const double *r, int k, const double *S, const double *R, double tol_pcg, int itmax_pcg,
                 double tau, int exit_rule, double xi, double *s, int *its);
int or_dacg_apply(int n, const int *rp, const int *ci, const double *v, const int *Lrp, const int *Lci,
                  const double *Lv, int m, const double *Qt, const double *x0, double tol, int itmax, double *x,
                  double *q_hist, int hist_cap);

static int bad = 0;
#define CHECK(c, ...)                    \
    do {                                 \
        if (!(c)) {                      \
            printf("FAIL: " __VA_ARGS__); \
            printf("\n");                \
            bad++;                       \
        }                                \
    } while (0)

/* 2-D 5-point Dirichlet Laplacian on an N x N grid (CSR, both triangles, sorted columns) */
static int lap2d(int N, int **rp, int **ci, double **v) {
    int n = N * N, k = 0;
    *rp = malloc(sizeof(int) * (n + 1));
    *ci = malloc(sizeof(int) * 5 * n);
    *v = malloc(sizeof(double) * 5 * n);
    for (int y = 0; y < N; y++)
        for (int x = 0; x < N; x++) {
            int i = x + N * y;
            (*rp)[i] = k;
            int c[5] = {i - N, i - 1, i, i + 1, i + N};
            int ok[5] = {y > 0, x > 0, 1, x < N - 1, y < N - 1};
            for (int t = 0; t < 5; t++)
                if (ok[t]) { (*ci)[k] = c[t]; (*v)[k] = (t == 2) ? 4.0 : -1.0; k++; }
        }
    (*rp)[n] = k;
    return n;
}

static double lcg(unsigned long long *s) {
    *s = *s * 6364136223846793005ULL + 1442695040888963407ULL;
    return ((*s >> 11) * (1.0 / 9007199254740992.0)) * 2.0 - 1.0;
}

static void defaults(or_opts *o, int p) {
    memset(o, 0, sizeof *o);
    o->p = p; o->itmax = 100; o->itmax_dacg = 5000; o->itmax_pcg = 20; o->kmax = 5; o->exit_rule = 1;
    o->tol = 1e-8; o->tol_dacg = 1e-2; o->tol_pcg = 1e-2; o->exit_xi = 0.1; o->shift0 = 1e-3; o->shift_max = 1.0;
    o->newton = 1; o->lfil = 30; o->tau_ic = 1e-2; o->jd_mmin = 5; o->jd_mmax = 10;
}

int main(void) {
    const int N = 12, p = 4;
    int *rp, *ci;
    double *v;
    int n = lap2d(N, &rp, &ci, &v);
    unsigned long long seed = 7;
    double *x0 = malloc(sizeof(double) * n * p);
    for (int i = 0; i < n * p; i++) x0[i] = lcg(&seed);
    /* closed form: 4 sin^2(i pi / 2(N+1)) + 4 sin^2(j pi / 2(N+1)), the four smallest */
    double mu[4];
    for (int t = 0; t < 4; t++) mu[t] = 4.0 * pow(sin((t + 1) * M_PI / (2.0 * (N + 1))), 2);
    double ref[4] = {2 * mu[0], mu[0] + mu[1], mu[0] + mu[1], 2 * mu[1]};
    double ev[4], *V = malloc(sizeof(double) * n * p), tr[8 * 400];
    or_stats st;
    or_opts o;
    const char *names[] = {"DACG-Newton", "full BFGS", "DACG alone", "IC(lfil, tau)", "Jacobi-Davidson"};
    for (int variant = 0; variant < 5; variant++) {
        defaults(&o, p);
        if (variant == 1) o.bfgs_full = 1;
        if (variant == 2) o.newton = 0;
        if (variant == 3) o.ict = 1;
        if (variant == 4) { o.jd = 1; o.jd_mmin = 2; o.jd_mmax = 4; }
        int rc = or_solve(n, rp, ci, v, &o, x0, ev, V, &st, tr, 400);
        CHECK(rc == 0, "%s rc %d", names[variant], rc);
        for (int t = 0; t < p; t++) CHECK(fabs(ev[t] - ref[t]) <= 1e-10 * ref[t], "%s eig %d", names[variant], t);
    }
    /* backward of sum(lambda) + sum v_1^2 */
    double ge[4] = {1, 1, 1, 1}, *gV = calloc((size_t)n * p, sizeof(double)), *gv = malloc(sizeof(double) * rp[n]);
    for (int i = 0; i < n; i++) gV[i] = 2 * V[i];
    CHECK(or_backward(n, rp, ci, v, p, ev, V, ge, gV, 1e-12, 2000, 1e-3, 1.0, gv) >= 0, "backward");
    /* factors and solves */
    int nl = or_tril_nnz(n, rp, ci);
    int *Lrp = malloc(sizeof(int) * (n + 1)), *Lci = malloc(sizeof(int) * nl);
    double *Lv = malloc(sizeof(double) * nl), sh;
    CHECK(or_ic0(n, rp, ci, v, 1e-3, 1.0, Lrp, Lci, Lv, &sh) == 0, "ic0");
    int *Trp, *Tci;
    double *Tv;
    CHECK(or_ict(n, rp, ci, v, 3, 1e-2, 1e-3, 1.0, &Trp, &Tci, &Tv, &sh) == 0, "ict");
    or_free(Trp); or_free(Tci); or_free(Tv);
    double *b = malloc(sizeof(double) * n), *x = malloc(sizeof(double) * n), *y = malloc(sizeof(double) * n);
    for (int i = 0; i < n; i++) b[i] = lcg(&seed);
    or_lsolve(n, Lrp, Lci, Lv, b, x);
    or_ltsolve(n, Lrp, Lci, Lv, x, y);
    or_spmv(n, rp, ci, v, y, x);
    /* BFGS apply, window, PCG and DACG entry points */
    const int k = 3;
    double *S = malloc(sizeof(double) * n * 5), *R = malloc(sizeof(double) * n * 5);
    for (int t = 0; t < 5; t++) {
        for (int i = 0; i < n; i++) S[t * n + i] = lcg(&seed);
        or_spmv(n, rp, ci, v, S + t * n, R + t * n);
        for (int i = 0; i < n; i++) R[t * n + i] = -R[t * n + i];
    }
    or_bfgspk_apply(n, Lrp, Lci, Lv, k, S, R, 1, V, b, x);
    CHECK(or_window_apply(n, Lrp, Lci, Lv, 2, 5, S, R, 1, V, b, x) == 2, "window");
    double *Au = malloc(sizeof(double) * n), *r = malloc(sizeof(double) * n);
    or_spmv(n, rp, ci, v, V, Au);
    double th = 0;
    for (int i = 0; i < n; i++) th += V[i] * Au[i];
    for (int i = 0; i < n; i++) r[i] = Au[i] - th * V[i];
    int its = 0;
    or_pcg_apply(n, rp, ci, v, Lrp, Lci, Lv, th, 1, V, V, Au, r, k, S, R, 1e-2, 20, 1e-8, 1, 0.1, x, &its);
    double qh[50];
    or_dacg_apply(n, rp, ci, v, Lrp, Lci, Lv, 1, V, x0 + n, 1e-6, 50, x, qh, 50);
    double H[9] = {2, 1, 0, 1, 3, 1, 0, 1, 4}, hev[3], Y[9];
    or_symeig(3, H, hev, Y);
    CHECK(hev[0] <= hev[1] && hev[1] <= hev[2], "symeig order");
    free(rp); free(ci); free(v); free(x0); free(V); free(gV); free(gv); free(Lrp); free(Lci); free(Lv);
    free(b); free(x); free(y); free(S); free(R); free(Au); free(r);
    printf("oracle driver: bad %d\n", bad);
    return bad != 0;
}
