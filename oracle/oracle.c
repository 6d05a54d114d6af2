/*
 * Oracle: a plain, slow, single-threaded FP64 CPU implementation of the
 * DACG-Newton eigensolver of Bergamaschi & Martinez, "Efficiently
 * preconditioned Inexact Newton methods for large symmetric eigenvalue
 * problems" (arXiv 1312.1553).
 *
 * THIS IS TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no code, header,
 * table or helper with the HIP library; both are fed the same seeded inputs.
 *
 * Paper references (section / algorithm / equation numbers of the paper):
 *   eq. (1.2)   Newton-Grassmann correction equation
 *   Sec. 2      projected IC initial preconditioner and the simplified BFGS
 *               update (eq. (2.2)), with y_k replaced by -r_k
 *   eq. (3.1)   normalised Newton step u_{k+1} = (u_k + s)/||u_k + s||
 *   Sec. 3.2    deflation: J_k and P_k projected against Q = [v_1..v_{j-1}, u_k]
 *   Sec. 4.1    DACG initial guess (algorithm only cited by the paper)
 *   Alg. 1      c = P_k g  (two loops around the IC solve, then CGS vs Q)
 *   Sec. 4.3    PCG for the correction equation and its exit tests (eq. (4.2))
 *   Sec. 4.4    k_max window; Alg. 2 (DACG-Newton driver)
 *
 * Readings where the paper is silent or ambiguous (listed in the design notes):
 *   r_k = A u_k - theta_k u_k and J_k s_k = -r_k (sign of r, Sec. 2 vs eq. (1.2));
 *   PCG starts from s = 0 with g_0 = -(I - QQ^T) r_k;
 *   J_k is applied literally with both projections;
 *   exit test (iii) uses the normalised x = (u+s)/||u+s||;
 *   exit test (iv) "eigen-residual decreases slower than ||g||" is read as
 *   ||g_l|| <= xi * eigres_l (exit_rule 1), or disabled (exit_rule 0);
 *   BFGS pairs are kept in chronological order, newest applied first in the
 *   first loop; a pair with alpha >= -1e-12 ||s|| ||r|| is not stored;
 *   the BFGS history restarts with each eigenpair (k := 0 in Alg. 2);
 *   IC(0) on the pattern of tril(A); on a non-positive pivot the factor is
 *   restarted on A + a*diag(A), a = shift0, 2*shift0, ... <= shift_max;
 *   IC(lfil, tau_IC): ILUT-style dual dropping on the diagonally scaled matrix
 *   (the rule is spelled out at or_ict);
 *   DACG is a preconditioned Fletcher-Reeves nonlinear CG on the Rayleigh
 *   quotient over the complement of the converged eigenvectors, with an exact
 *   line search (closed-form minimiser of q(x + a d));
 *   when the Newton phase stalls (a PCG solve takes no step, or the outer
 *   residual fails to drop below 0.9x in two consecutive steps) the start was
 *   not close enough in the sense of Sec. 4.1: DACG is resumed from the current
 *   iterate to 0.005 ||r||/theta (within [tol, tol_DACG]), the BFGS history is
 *   restarted, and Newton continues (at most 5 times per eigenpair).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#define OR_MAXP 32

typedef struct {
    int p, itmax, itmax_dacg, itmax_pcg, kmax, exit_rule;
    double tol, tol_dacg, tol_pcg, exit_xi, shift0, shift_max;
    int newton; /* 1: DACG-Newton (Alg. 2); 0: DACG alone to tol, the DACG rows of Tables 4, 5, 7 and 8 */
    int bfgs_full; /* 0: pairs (s_k, r_k) of eq. (2.2), y_k ~ -r_k; 1: y_k = r_{k+1} - r_k of eq. (2.1), stored
                      as (s_k, r_k - r_{k+1}) so that Alg. 1 applies unchanged */
    int ict;       /* 0: IC(0) on the pattern of tril(A); 1: IC(lfil, tau_ic) of Sec. 2 (or_ict) */
    int lfil;
    double tau_ic;
    int jd;        /* 1: Jacobi-Davidson outer iteration (Sec. 6) in place of DACG + Newton, with the same PCG
                      (and the BFGS pairs when kmax > 0) as the correction solver */
    int jd_mmin, jd_mmax; /* restart and maximum dimensions of the search space (5 and 10 in Sec. 6) */
} or_opts;

typedef struct {
    int dacg_its[OR_MAXP], outer_its[OR_MAXP], pcg_its[OR_MAXP], converged[OR_MAXP];
    double relres[OR_MAXP];
    long long mvp_dacg, mvp_newton;
    int bfgs_skipped, pcg_breakdowns, ntrace, status;
    double shift_used, t_factor, t_dacg, t_newton;
    int dacg_restarts;
    long long nnz_L; /* entries of the factor L, diagonal included */
    double fill;     /* sigma of Sec. 5: nnz(L) / nnz(tril(A)) */
} or_stats;

static double now_s(void) {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return ts.tv_sec + 1e-9 * ts.tv_nsec;
}

/* ---------------------------------------------------------------- vectors */
static double dot(int n, const double *x, const double *y) {
    double s = 0.0;
    for (int i = 0; i < n; i++) s += x[i] * y[i];
    return s;
}
static double nrm2(int n, const double *x) { return sqrt(dot(n, x, x)); }
static void axpy(int n, double a, const double *x, double *y) {
    for (int i = 0; i < n; i++) y[i] += a * x[i];
}
static void scal(int n, double a, double *x) {
    for (int i = 0; i < n; i++) x[i] *= a;
}
static void copy(int n, const double *x, double *y) { memcpy(y, x, sizeof(double) * (size_t)n); }

/* ---------------------------------------------------------------- matrix */
/* y = A x for A in CSR. */
void or_spmv(int n, const int *rp, const int *ci, const double *v, const double *x, double *y) {
    for (int i = 0; i < n; i++) {
        double s = 0.0;
        for (int e = rp[i]; e < rp[i + 1]; e++) s += v[e] * x[ci[e]];
        y[i] = s;
    }
}

/* Number of stored entries of tril(A) (the IC(0) pattern). */
int or_tril_nnz(int n, const int *rp, const int *ci) {
    int c = 0;
    for (int i = 0; i < n; i++)
        for (int e = rp[i]; e < rp[i + 1]; e++) c += (ci[e] <= i);
    return c;
}

/*
 * IC(0) factor L (L L^T = A on the pattern of tril(A)), Sec. 2: the initial
 * preconditioner P0^ = (L L^T)^{-1}.  Row-by-row ("up-looking"):
 *   L_ij = (A_ij - sum_{m<j} L_im L_jm) / L_jj   for (i,j) in tril pattern, j<i
 *   L_ii = sqrt(A_ii - sum_{m<i} L_im^2)
 * A pivot <= 0 restarts on A + a*diag(A).  Output rows keep the column order
 * of A, so the diagonal is last.  Returns 0, or -1 when no shift up to
 * shift_max gives positive pivots.
 */
int or_ic0(int n, const int *rp, const int *ci, const double *v, double shift0, double shift_max,
           int *Lrp, int *Lci, double *Lv, double *shift_used) {
    /* copy the pattern of tril(A) */
    Lrp[0] = 0;
    for (int i = 0; i < n; i++) {
        int c = Lrp[i];
        for (int e = rp[i]; e < rp[i + 1]; e++)
            if (ci[e] <= i) Lci[c++] = ci[e];
        Lrp[i + 1] = c;
        if (c == Lrp[i] || Lci[c - 1] != i) return -2; /* missing diagonal */
    }
    double a = 0.0;
    for (;;) {
        int ok = 1;
        for (int i = 0; i < n && ok; i++) {
            int c = Lrp[i];
            for (int e = rp[i]; e < rp[i + 1]; e++) {
                int j = ci[e];
                if (j > i) continue;
                double aij = v[e];
                if (j == i) {
                    aij *= (1.0 + a);
                    double d = aij;
                    for (int t = Lrp[i]; t < c; t++) d -= Lv[t] * Lv[t];
                    if (!(d > 0.0)) { ok = 0; break; }
                    Lv[c] = sqrt(d);
                } else {
                    /* sum over m < j present in both row i (entries so far) and row j */
                    double s = aij;
                    int p = Lrp[i], q = Lrp[j];
                    int pend = c, qend = Lrp[j + 1] - 1; /* exclude the diagonal of row j */
                    while (p < pend && q < qend) {
                        if (Lci[p] == Lci[q]) { s -= Lv[p] * Lv[q]; p++; q++; }
                        else if (Lci[p] < Lci[q]) p++;
                        else q++;
                    }
                    Lv[c] = s / Lv[Lrp[j + 1] - 1];
                }
                c++;
            }
        }
        if (ok) break;
        a = (a == 0.0) ? shift0 : 2.0 * a;
        if (a > shift_max || shift0 <= 0.0) return -1;
    }
    if (shift_used) *shift_used = a;
    return 0;
}

/*
 * IC(lfil, tau_IC) factor, Sec. 2: the paper's own initial preconditioner, an
 * incomplete Cholesky factor with at most lfil entries off the diagonal in each
 * row of L and small entries dropped below the threshold tau_IC.  The paper
 * names only the two parameters; the dual dropping rule taken here follows
 * ILUT, row by row:
 *   the factor Ls is computed for the diagonally scaled matrix As = D^-1/2 A D^-1/2
 *   (D = diag(A), As_ij = (a_ij r_i) r_j with r_i = 1/sqrt(a_ii), diagonal included),
 *   so that the drop rule does not depend on the scaling of A, and returned as
 *   L = D^1/2 Ls (row i of Ls times sqrt(a_ii));
 *   row i: tau_i = tau_IC ||As(i,:)||_2 (the whole row, summed in column order);
 *   w = strictly lower part of row i of As; for k ascending over the nonzeros of
 *   w, fill included: l = w_k / Ls_kk; if |l| < tau_i the entry is dropped and
 *   takes no part in the elimination, else it is a candidate Ls_ik = l and
 *   w_m -= l Ls_mk for every earlier row m > k holding an entry in column k
 *   (which may create fill at m);
 *   of the candidates the lfil largest in magnitude are kept (ties go to the
 *   smaller column); Ls_ii = sqrt(As_ii - sum of the kept Ls_ik^2 in column order);
 *   a pivot <= 0 restarts the whole factorisation, scaling and thresholds
 *   included, on A + a diag(A) (diagonal a_ii (1 + a)), a = shift0, 2 shift0, ...
 *   <= shift_max.
 * With tau_IC = 0 and lfil >= n - 1 this is the exact Cholesky factor.
 * Output: CSR of L (columns ascending, diagonal last) in arrays allocated here
 * (release each with or_free).  Returns 0, -1 when no shift up to shift_max
 * gives positive pivots, -2 for a missing or non-positive diagonal or lfil < 0.
 */
typedef struct { int col; double val; } ict_ent;

static int ict_by_size(const void *a, const void *b) {
    const ict_ent *x = a, *y = b;
    double ax = fabs(x->val), ay = fabs(y->val);
    if (ax != ay) return ax > ay ? -1 : 1;
    return x->col - y->col;
}

static int ict_by_col(const void *a, const void *b) {
    return ((const ict_ent *)a)->col - ((const ict_ent *)b)->col;
}

void or_free(void *p) { free(p); }

int or_ict(int n, const int *rp, const int *ci, const double *v, int lfil, double tau, double shift0,
           double shift_max, int **Lrp_out, int **Lci_out, double **Lv_out, double *shift_used) {
    size_t N = (size_t)n;
    if (lfil < 0) return -2;
    double *dg = malloc(sizeof(double) * N);
    for (int i = 0; i < n; i++) {
        dg[i] = 0.0;
        for (int e = rp[i]; e < rp[i + 1]; e++)
            if (ci[e] == i) dg[i] = v[e];
        if (!(dg[i] > 0.0)) { free(dg); return -2; }
    }
    double *r = malloc(sizeof(double) * N), *sq = malloc(sizeof(double) * N), *taui = malloc(sizeof(double) * N);
    double *ds = malloc(sizeof(double) * N); /* diagonal of As */
    double *w = calloc(N, sizeof(double));
    int *inw = malloc(sizeof(int) * N);   /* position m holds a pending entry of the current row */
    int *list = malloc(sizeof(int) * N);  /* pending positions of the current row, ascending */
    ict_ent *cand = malloc(sizeof(ict_ent) * N);
    int *head = malloc(sizeof(int) * N), *tail = malloc(sizeof(int) * N); /* column lists of Ls */
    size_t cap = (size_t)rp[n] + N;
    int *Lrp = malloc(sizeof(int) * (N + 1));
    int *Lci = malloc(sizeof(int) * cap), *Lrow = malloc(sizeof(int) * cap), *nxt = malloc(sizeof(int) * cap);
    double *Lv = malloc(sizeof(double) * cap);
    double a = 0.0;
    int rc = 0;
    for (;;) {
        /* scaling of the matrix factored in this attempt, A + a diag(A) */
        for (int i = 0; i < n; i++) {
            double d = dg[i] * (1.0 + a);
            sq[i] = sqrt(d);
            r[i] = 1.0 / sq[i];
            ds[i] = d * r[i] * r[i];
        }
        for (int i = 0; i < n; i++) {
            double s2 = 0.0;
            for (int e = rp[i]; e < rp[i + 1]; e++) {
                double as = ci[e] == i ? ds[i] : v[e] * r[i] * r[ci[e]];
                s2 += as * as;
            }
            taui[i] = tau * sqrt(s2);
        }
        for (int i = 0; i < n; i++) { inw[i] = 0; head[i] = tail[i] = -1; }
        size_t nz = 0;
        int ok = 1;
        Lrp[0] = 0;
        for (int i = 0; i < n && ok; i++) {
            int len = 0;
            for (int e = rp[i]; e < rp[i + 1]; e++) {
                int j = ci[e];
                if (j >= i) continue;
                w[j] = v[e] * r[i] * r[j];
                inw[j] = 1;
                list[len++] = j; /* the columns of a CSR row ascend */
            }
            int nc = 0;
            for (int t = 0; t < len; t++) {
                int k = list[t];
                double l = w[k] / Lv[Lrp[k + 1] - 1];
                w[k] = 0.0;
                inw[k] = 0;
                if (fabs(l) < taui[i]) continue;
                cand[nc].col = k;
                cand[nc].val = l;
                nc++;
                for (int e = head[k]; e >= 0; e = nxt[e]) {
                    int m = Lrow[e];
                    if (!inw[m]) { /* fill: insert m into the ascending tail of the list */
                        int p = len++;
                        while (p > t + 1 && list[p - 1] > m) { list[p] = list[p - 1]; p--; }
                        list[p] = m;
                        inw[m] = 1;
                    }
                    w[m] -= l * Lv[e];
                }
            }
            if (nc > lfil) {
                qsort(cand, (size_t)nc, sizeof(ict_ent), ict_by_size);
                nc = lfil;
                qsort(cand, (size_t)nc, sizeof(ict_ent), ict_by_col);
            }
            double d = ds[i];
            for (int t = 0; t < nc; t++) d -= cand[t].val * cand[t].val;
            if (!(d > 0.0)) { ok = 0; break; }
            if (nz + (size_t)nc + 1 > cap) {
                cap = 2 * cap + (size_t)nc + 1;
                Lci = realloc(Lci, sizeof(int) * cap);
                Lrow = realloc(Lrow, sizeof(int) * cap);
                nxt = realloc(nxt, sizeof(int) * cap);
                Lv = realloc(Lv, sizeof(double) * cap);
            }
            for (int t = 0; t < nc; t++) {
                int k = cand[t].col;
                Lci[nz] = k;
                Lrow[nz] = i;
                Lv[nz] = cand[t].val;
                nxt[nz] = -1;
                if (tail[k] < 0) head[k] = (int)nz;
                else nxt[tail[k]] = (int)nz;
                tail[k] = (int)nz;
                nz++;
            }
            Lci[nz] = i;
            Lrow[nz] = i;
            Lv[nz] = sqrt(d);
            nxt[nz] = -1;
            nz++;
            Lrp[i + 1] = (int)nz;
        }
        if (ok) break;
        a = (a == 0.0) ? shift0 : 2.0 * a;
        if (a > shift_max || shift0 <= 0.0) { rc = -1; break; }
    }
    if (rc == 0) {
        for (int i = 0; i < n; i++)
            for (int e = Lrp[i]; e < Lrp[i + 1]; e++) Lv[e] *= sq[i];
        *Lrp_out = Lrp;
        *Lci_out = Lci;
        *Lv_out = Lv;
        if (shift_used) *shift_used = a;
    } else {
        free(Lrp); free(Lci); free(Lv);
    }
    free(Lrow); free(nxt); free(dg); free(ds); free(r); free(sq); free(taui); free(w); free(inw); free(list); free(cand);
    free(head); free(tail);
    return rc;
}

/* Forward substitution L x = b (L rows, diagonal last). */
void or_lsolve(int n, const int *Lrp, const int *Lci, const double *Lv, const double *b, double *x) {
    for (int i = 0; i < n; i++) {
        double s = b[i];
        int d = Lrp[i + 1] - 1;
        for (int e = Lrp[i]; e < d; e++) s -= Lv[e] * x[Lci[e]];
        x[i] = s / Lv[d];
    }
}

/* Back substitution L^T x = b using the rows of L (column-oriented sweep). */
void or_ltsolve(int n, const int *Lrp, const int *Lci, const double *Lv, const double *b, double *x) {
    copy(n, b, x);
    for (int i = n - 1; i >= 0; i--) {
        int d = Lrp[i + 1] - 1;
        x[i] /= Lv[d];
        for (int e = Lrp[i]; e < d; e++) x[Lci[e]] -= Lv[e] * x[i];
    }
}

/* ------------------------------------------------------ problem context */
typedef struct {
    int n;
    const int *rp, *ci;
    const double *v;
    const int *Lrp, *Lci;
    const double *Lv;
    double *tmp; /* n scratch for the IC solve */
} prob;

/* c = (L L^T)^{-1} w */
static void ic_apply(const prob *P, const double *w, double *c) {
    or_lsolve(P->n, P->Lrp, P->Lci, P->Lv, w, P->tmp);
    or_ltsolve(P->n, P->Lrp, P->Lci, P->Lv, P->tmp, c);
}

/* x -= Q (Q^T x), classical Gram-Schmidt against the m rows of Q (m x n). */
static void cgs(int n, int m, const double *Q, double *x, double *z) {
    for (int j = 0; j < m; j++) z[j] = dot(n, Q + (size_t)j * n, x);
    for (int j = 0; j < m; j++) axpy(n, -z[j], Q + (size_t)j * n, x);
}

/*
 * Alg. 1 (Sec. 4.2): c = P_k g for the BFGS-updated preconditioner, eq. (2.2)
 * applied recursively k times to P0^, then CGS against Q.  S and R hold the k
 * stored pairs as rows (k x n), oldest first; alpha[s] = s_s^T r_s.
 *   w := g; for s = k-1..0: a_s = s_s^T w / alpha_s; w -= a_s r_s
 *   c := P0^ w
 *   for s = 0..k-1: b = r_s^T c / alpha_s; c -= (a_s + b) s_s
 *   z := Q^T c; c -= Q z
 */
void or_bfgspk(const prob *P, int k, const double *S, const double *R, const double *alpha,
               int m, const double *Q, const double *g, double *c, double *w, double *a, double *z) {
    int n = P->n;
    copy(n, g, w);
    for (int s = k - 1; s >= 0; s--) {
        a[s] = dot(n, S + (size_t)s * n, w) / alpha[s];
        axpy(n, -a[s], R + (size_t)s * n, w);
    }
    ic_apply(P, w, c);
    for (int s = 0; s < k; s++) {
        double b = dot(n, R + (size_t)s * n, c) / alpha[s];
        axpy(n, -(a[s] + b), S + (size_t)s * n, c);
    }
    cgs(n, m, Q, c, z);
}

/* y = J p = (I - QQ^T)(A - theta I)(I - QQ^T) p, written out literally (Sec. 3.2).
 * Also returns Ap_proj = A (I - QQ^T) p, used for the running t = A s. */
static void japply(const prob *P, double theta, int m, const double *Q, const double *p,
                   double *pp, double *Ap, double *y, double *z) {
    int n = P->n;
    copy(n, p, pp);
    cgs(n, m, Q, pp, z);
    or_spmv(n, P->rp, P->ci, P->v, pp, Ap);
    for (int i = 0; i < n; i++) y[i] = Ap[i] - theta * pp[i];
    cgs(n, m, Q, y, z);
}

enum { PCG_EXIT_MAXIT = 0, PCG_EXIT_TOL = 1, PCG_EXIT_EIGRES = 2, PCG_EXIT_STAG = 3, PCG_EXIT_BREAKDOWN = 4 };

/*
 * PCG on the correction equation J_k s = -r_k, s orthogonal to Q (Sec. 4.3),
 * with the preconditioner of Alg. 1 and the exit tests of Sec. 4.3:
 *  (i)   ||g_l|| <= tol_pcg ||g_0||
 *  (ii)  l = itmax_pcg
 *  (iii) ||A x - q(x) x|| < tau q(x),  x = (u + s_l)/||u + s_l||   (eq. (4.2))
 *  (iv)  exit_rule 1: ||g_l|| <= xi * eigres_l
 * Q holds m rows; row m-1 is u.  Au is A u.  Returns the exit reason.
 * work must hold 9 n doubles.
 */
int or_pcg(const prob *P, double theta, int m, const double *Q, const double *u, const double *Au,
           const double *r, int k, const double *S, const double *R, const double *alpha,
           double tol_pcg, int itmax_pcg, double tau, int exit_rule, double xi,
           double *s, int *its_out, double *work) {
    int n = P->n;
    double *g = work, *c = work + n, *p = work + 2 * (size_t)n, *y = work + 3 * (size_t)n;
    double *pp = work + 4 * (size_t)n, *Ap = work + 5 * (size_t)n, *t = work + 6 * (size_t)n;
    double *bw = work + 7 * (size_t)n, *x = work + 8 * (size_t)n;
    double z[OR_MAXP + 1], a[64];
    int reason = PCG_EXIT_MAXIT, its = 0;

    for (int i = 0; i < n; i++) { s[i] = 0.0; t[i] = 0.0; g[i] = -r[i]; }
    cgs(n, m, Q, g, z); /* g_0 = -(I - QQ^T) r */
    double g0 = nrm2(n, g);
    or_bfgspk(P, k, S, R, alpha, m, Q, g, c, bw, a, z);
    double rho = dot(n, g, c);
    copy(n, c, p);
    for (int l = 1; l <= itmax_pcg; l++) {
        japply(P, theta, m, Q, p, pp, Ap, y, z);
        double pJp = dot(n, p, y);
        if (!(pJp > 0.0)) { reason = PCG_EXIT_BREAKDOWN; break; }
        double gamma = rho / pJp;
        axpy(n, gamma, p, s);
        axpy(n, -gamma, y, g);
        axpy(n, gamma, Ap, t);
        its = l;
        double gn = nrm2(n, g);
        /* eigen-residual of x = (u+s)/||u+s||, with A(u+s) = Au + t */
        for (int i = 0; i < n; i++) x[i] = u[i] + s[i];
        double xx = dot(n, x, x);
        double xAx = 0.0;
        for (int i = 0; i < n; i++) xAx += x[i] * (Au[i] + t[i]);
        double q = xAx / xx;
        double e2 = 0.0;
        for (int i = 0; i < n; i++) {
            double d = Au[i] + t[i] - q * x[i];
            e2 += d * d;
        }
        double eigres = sqrt(e2 / xx);
        if (gn <= tol_pcg * g0) { reason = PCG_EXIT_TOL; break; }
        if (eigres < tau * q) { reason = PCG_EXIT_EIGRES; break; }
        if (exit_rule == 1 && gn <= xi * eigres) { reason = PCG_EXIT_STAG; break; }
        if (l == itmax_pcg) break;
        or_bfgspk(P, k, S, R, alpha, m, Q, g, c, bw, a, z);
        double rho1 = dot(n, g, c);
        double beta = rho1 / rho;
        for (int i = 0; i < n; i++) p[i] = c[i] + beta * p[i];
        rho = rho1;
    }
    *its_out = its;
    return reason;
}

/*
 * Minimiser over a of q(x + a d) = (xAx + 2 a dAx + a^2 dAd) / (xx + 2 a xd + a^2 dd).
 * Setting dq/da = 0 gives  A2 a^2 + B2 a + C2 = 0  with
 *   A2 = dAd*xd - dAx*dd,  B2 = dAd*xx - xAx*dd,  C2 = dAx*xx - xAx*xd.
 * Both roots are evaluated and the one with the smaller quotient is taken.
 */
double or_linesearch(double xAx, double dAx, double dAd, double xx, double xd, double dd) {
    double A2 = dAd * xd - dAx * dd, B2 = dAd * xx - xAx * dd, C2 = dAx * xx - xAx * xd;
    double r1, r2;
    if (A2 == 0.0) {
        r1 = r2 = (B2 != 0.0) ? -C2 / B2 : 0.0;
    } else {
        double disc = B2 * B2 - 4.0 * A2 * C2;
        if (disc < 0.0) disc = 0.0;
        double tq = -0.5 * (B2 + (B2 >= 0.0 ? 1.0 : -1.0) * sqrt(disc));
        r1 = tq / A2;
        r2 = (tq != 0.0) ? C2 / tq : r1;
    }
    double q1 = (xAx + 2 * r1 * dAx + r1 * r1 * dAd) / (xx + 2 * r1 * xd + r1 * r1 * dd);
    double q2 = (xAx + 2 * r2 * dAx + r2 * r2 * dAd) / (xx + 2 * r2 * xd + r2 * r2 * dd);
    return (q2 < q1) ? r2 : r1;
}

/*
 * DACG (Sec. 4.1; the paper cites the method): preconditioned nonlinear CG
 * minimising q(x) = x'Ax/x'x over the complement of the m rows of Qt.
 *   g = A x - q x ; stop when ||g|| <= tol q (x normalised)
 *   h = (I - Qt Qt^T) P0^ g ; gamma = g^T h
 *   d = -h + (gamma / gamma_prev) d      (Fletcher-Reeves; d = -h first)
 *   x <- (x + a d)/||x + a d|| with a the exact minimiser of q along d
 * A x is updated through A d (one SpMV per step).  q_hist (if not NULL)
 * receives q after each step.  Returns the number of steps; mvp counts SpMVs.
 */
int or_dacg(const prob *P, int m, const double *Qt, const double *x0, double tol, int itmax,
            double *x, double *q_hist, int hist_cap, long long *mvp, double *work) {
    int n = P->n;
    double *Ax = work, *g = work + n, *h = work + 2 * (size_t)n, *d = work + 3 * (size_t)n;
    double *Ad = work + 4 * (size_t)n;
    double z[OR_MAXP + 1];
    copy(n, x0, x);
    cgs(n, m, Qt, x, z);
    cgs(n, m, Qt, x, z);
    scal(n, 1.0 / nrm2(n, x), x);
    or_spmv(n, P->rp, P->ci, P->v, x, Ax);
    (*mvp)++;
    double q = dot(n, x, Ax);
    double gamma_prev = 0.0;
    int it = 0;
    for (int i = 0; i < n; i++) d[i] = 0.0; /* no previous direction: the first step is d = -h */
    for (; it < itmax; it++) {
        for (int i = 0; i < n; i++) g[i] = Ax[i] - q * x[i];
        if (nrm2(n, g) <= tol * q) break;
        ic_apply(P, g, h);
        cgs(n, m, Qt, h, z);
        double gamma = dot(n, g, h);
        double beta = (it == 0 || gamma_prev == 0.0) ? 0.0 : gamma / gamma_prev;
        for (int i = 0; i < n; i++) d[i] = -h[i] + beta * d[i];
        or_spmv(n, P->rp, P->ci, P->v, d, Ad);
        (*mvp)++;
        double xx = dot(n, x, x), xAx = dot(n, x, Ax), dAx = dot(n, d, Ax), dAd = dot(n, d, Ad);
        double xd = dot(n, x, d), dd = dot(n, d, d);
        double a = or_linesearch(xAx, dAx, dAd, xx, xd, dd);
        axpy(n, a, d, x);
        axpy(n, a, Ad, Ax);
        double nx = nrm2(n, x);
        scal(n, 1.0 / nx, x);
        scal(n, 1.0 / nx, Ax);
        q = dot(n, x, Ax);
        if (q_hist && it < hist_cap) q_hist[it] = q;
        gamma_prev = gamma;
    }
    return it;
}

/* --------------------------------------------------------------- driver */
typedef struct {
    int k, kmax, n;
    double *S, *R; /* kmax x n, row 0 = oldest */
    double alpha[64];
} pairs_t;

/* k_max window (Sec. 4.4): append (s, r); when full, drop the oldest. */
static void pairs_push(pairs_t *W, const double *s, const double *r, double alpha) {
    int n = W->n;
    if (W->kmax <= 0) return;
    if (W->k == W->kmax) {
        memmove(W->S, W->S + n, sizeof(double) * (size_t)n * (W->kmax - 1));
        memmove(W->R, W->R + n, sizeof(double) * (size_t)n * (W->kmax - 1));
        memmove(W->alpha, W->alpha + 1, sizeof(double) * (W->kmax - 1));
        W->k--;
    }
    copy(n, s, W->S + (size_t)W->k * n);
    copy(n, r, W->R + (size_t)W->k * n);
    W->alpha[W->k] = alpha;
    W->k++;
}

/*
 * Eigen-decomposition of a symmetric m x m matrix H (row-major, overwritten) by the
 * cyclic Jacobi method: rotations annihilate each off-diagonal entry in turn until
 * the off-diagonal mass is below 1e-30 of the total.  ev[0..m-1] ascending, Y
 * column-major (column c = eigenvector of ev[c]).  Used for the Rayleigh-Ritz step.
 */
void or_symeig(int m, double *H, double *ev, double *Y) {
    for (int i = 0; i < m; i++)
        for (int c = 0; c < m; c++) Y[c * m + i] = (i == c);
    for (int sweep = 0; sweep < 100; sweep++) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < m; i++)
            for (int c = 0; c < m; c++) {
                tot += H[i * m + c] * H[i * m + c];
                if (i != c) off += H[i * m + c] * H[i * m + c];
            }
        if (off <= 1e-30 * tot) break;
        for (int a = 0; a < m - 1; a++)
            for (int b = a + 1; b < m; b++) {
                double hab = H[a * m + b];
                if (hab == 0.0) continue;
                /* rotation angle that zeroes H[a][b]: tan(2 phi) = 2 h_ab / (h_bb - h_aa) */
                double zeta = (H[b * m + b] - H[a * m + a]) / (2.0 * hab);
                double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                double cs = 1.0 / sqrt(1.0 + t * t), sn = t * cs;
                for (int k = 0; k < m; k++) { /* H <- H G (columns a, b) */
                    double x = H[k * m + a], y = H[k * m + b];
                    H[k * m + a] = cs * x - sn * y;
                    H[k * m + b] = sn * x + cs * y;
                }
                for (int k = 0; k < m; k++) { /* H <- G^T H (rows a, b) */
                    double x = H[a * m + k], y = H[b * m + k];
                    H[a * m + k] = cs * x - sn * y;
                    H[b * m + k] = sn * x + cs * y;
                }
                for (int k = 0; k < m; k++) { /* Y <- Y G */
                    double x = Y[a * m + k], y = Y[b * m + k];
                    Y[a * m + k] = cs * x - sn * y;
                    Y[b * m + k] = sn * x + cs * y;
                }
            }
    }
    for (int i = 0; i < m; i++) ev[i] = H[i * m + i];
    /* ascending order (insertion sort of the pairs) */
    for (int a = 1; a < m; a++)
        for (int b = a; b > 0 && ev[b] < ev[b - 1]; b--) {
            double t = ev[b]; ev[b] = ev[b - 1]; ev[b - 1] = t;
            for (int k = 0; k < m; k++) {
                double y = Y[b * m + k]; Y[b * m + k] = Y[(b - 1) * m + k]; Y[(b - 1) * m + k] = y;
            }
        }
}

/*
 * Jacobi-Davidson for eigenpair j (Sec. 6; readings in the design notes): the
 * search space V (orthonormal, orthogonal to v_1..v_{j-1}) starts from x0;
 * each step takes the Ritz pair (theta, u) of the smallest Ritz value from
 * H = V^T A V, tests ||A u - theta u|| <= tau theta, restarts V with the m_min
 * smallest Ritz vectors when it holds m_max vectors, and expands V with the
 * correction s of J s = -r from the PCG of Sec. 4.3 (with the BFGS pairs of
 * the correction solves when kmax > 0).  When the PCG takes no step (J is
 * indefinite far from the eigenvalue) the space grows by its first
 * preconditioned direction instead.  The Ritz vector is left in
 * Qm + j n; returns the number of outer steps.
 */
static int jd_pair(const prob *P, const or_opts *o, int j, double *Qm, const double *x0, pairs_t *W, or_stats *st,
                   double *theta_out, double *rn_out, double *work, double *Au, double *r, double *s, double *trace,
                   int trace_cap) {
    int n = P->n;
    size_t N = (size_t)n;
    int mmax = o->jd_mmax, mmin = o->jd_mmin;
    double *V = malloc(sizeof(double) * N * mmax), *AV = malloc(sizeof(double) * N * mmax);
    double *T2 = malloc(sizeof(double) * N * mmax);
    double *t = malloc(sizeof(double) * N);
    double *H = calloc((size_t)mmax * mmax, sizeof(double)), *Hw = malloc(sizeof(double) * mmax * mmax);
    double *Y = malloc(sizeof(double) * mmax * mmax), ev[64], z[OR_MAXP + 64];
    double *u = Qm + (size_t)j * N;
    double theta = 0.0, rn = 0.0;
    int m = 0, k = 0;
    W->k = 0;
    copy(n, x0, t);
    for (;;) {
        /* expand: t orthogonal to v_1..v_{j-1} and to V (classical Gram-Schmidt, twice), normalised */
        for (int pass = 0; pass < 2; pass++) {
            cgs(n, j, Qm, t, z);
            cgs(n, m, V, t, z);
        }
        double tn = nrm2(n, t);
        if (!(tn > 0.0)) break;
        scal(n, 1.0 / tn, t);
        copy(n, t, V + (size_t)m * N);
        or_spmv(n, P->rp, P->ci, P->v, t, AV + (size_t)m * N);
        st->mvp_newton++;
        for (int i = 0; i <= m; i++) {
            double h = dot(n, V + (size_t)i * N, AV + (size_t)m * N);
            H[i * mmax + m] = h;
            H[m * mmax + i] = h;
        }
        m++;
        /* Rayleigh-Ritz: smallest Ritz pair of H */
        for (int a = 0; a < m; a++)
            for (int b = 0; b < m; b++) Hw[a * m + b] = H[a * mmax + b];
        or_symeig(m, Hw, ev, Y);
        theta = ev[0];
        for (int i = 0; i < n; i++) { u[i] = 0.0; Au[i] = 0.0; }
        for (int c = 0; c < m; c++) {
            axpy(n, Y[c], V + (size_t)c * N, u);
            axpy(n, Y[c], AV + (size_t)c * N, Au);
        }
        for (int i = 0; i < n; i++) r[i] = Au[i] - theta * u[i];
        rn = nrm2(n, r);
        if (trace && st->ntrace < trace_cap) {
            double *T = trace + 8 * (size_t)st->ntrace++;
            T[0] = j; T[1] = k; T[2] = theta; T[3] = rn; T[4] = m; T[5] = ev[m > 1 ? 1 : 0]; T[6] = 0.0; T[7] = 0.0;
        }
        if (rn <= o->tol * theta || k >= o->itmax) break;
        if (m == mmax) { /* thick restart with the m_min smallest Ritz vectors */
            for (int c = 0; c < mmin; c++) {
                double *tc = T2 + (size_t)c * N;
                for (int i = 0; i < n; i++) tc[i] = 0.0;
                for (int a = 0; a < m; a++) axpy(n, Y[c * m + a], V + (size_t)a * N, tc);
            }
            memcpy(V, T2, sizeof(double) * N * mmin);
            for (int c = 0; c < mmin; c++) {
                double *tc = T2 + (size_t)c * N;
                for (int i = 0; i < n; i++) tc[i] = 0.0;
                for (int a = 0; a < m; a++) axpy(n, Y[c * m + a], AV + (size_t)a * N, tc);
            }
            memcpy(AV, T2, sizeof(double) * N * mmin);
            for (int a = 0; a < mmax * mmax; a++) H[a] = 0.0;
            for (int c = 0; c < mmin; c++) H[c * mmax + c] = ev[c];
            m = mmin;
        }
        /* correction equation, Sec. 4.3 PCG with the same exit tests */
        int its = 0;
        int why = or_pcg(P, theta, j + 1, Qm, u, Au, r, W->k, W->S, W->R, W->alpha, o->tol_pcg, o->itmax_pcg,
                         o->tol, o->exit_rule, o->exit_xi, s, &its, work);
        if (why == PCG_EXIT_BREAKDOWN) st->pcg_breakdowns++;
        st->pcg_its[j] += its;
        st->mvp_newton += its;
        if (its > 0) {
            double alpha = dot(n, s, r), sn2 = dot(n, s, s);
            if (alpha < -1e-12 * sqrt(sn2) * rn) pairs_push(W, s, r, alpha);
            else st->bfgs_skipped++;
            copy(n, s, t);
        } else {
            copy(n, work + 2 * N, t); /* the PCG's first direction: preconditioned projected residual */
        }
        k++;
    }
    free(V); free(AV); free(T2); free(t); free(H); free(Hw); free(Y);
    *theta_out = theta;
    *rn_out = rn;
    return k;
}

/*
 * Alg. 2 (DACG-Newton).  A in CSR (both triangles), x0 = p x n starting block
 * (row j for eigenpair j+1).  Outputs evals[p] ascending and evecs (p x n,
 * row j = v_{j+1}) with the first entry above 1e-12 ||v||_inf made positive.
 * trace (optional, trace_cap records of 8 doubles) receives per outer step:
 *   j, k, theta_k, ||r_k||, alpha_k = s_k^T r_k, ||s_k||^2, theta_{k+1}, PCG its;
 *   per return to DACG from a stalled Newton phase (k recorded as -1):
 *   j, -1, DACG tolerance, DACG its, theta and ||r|| after, theta and ||r|| before;
 *   with jd = 1, per Rayleigh-Ritz step: j, k, theta, ||r||, dim V, second Ritz value, 0, 0.
 * Returns 0 when every pair converged, 1 if some did not, <0 on errors.
 */
int or_solve(int n, const int *rp, const int *ci, const double *v, const or_opts *o,
             const double *x0, double *evals, double *evecs, or_stats *st, double *trace, int trace_cap) {
    memset(st, 0, sizeof(*st));
    int p = o->p;
    if (p < 1 || p > OR_MAXP || n < 1) return -1;
    double t0 = now_s();
    int nnzL = or_tril_nnz(n, rp, ci);
    int *Lrp, *Lci;
    double *Lv;
    int rc;
    if (o->ict) {
        rc = or_ict(n, rp, ci, v, o->lfil, o->tau_ic, o->shift0, o->shift_max, &Lrp, &Lci, &Lv, &st->shift_used);
        if (rc != 0) { st->status = rc; return -2; }
    } else {
        Lrp = malloc(sizeof(int) * (size_t)(n + 1));
        Lci = malloc(sizeof(int) * (size_t)nnzL);
        Lv = malloc(sizeof(double) * (size_t)nnzL);
        rc = or_ic0(n, rp, ci, v, o->shift0, o->shift_max, Lrp, Lci, Lv, &st->shift_used);
        if (rc != 0) { free(Lrp); free(Lci); free(Lv); st->status = rc; return -2; }
    }
    st->nnz_L = Lrp[n];
    st->fill = (double)Lrp[n] / (double)nnzL;
    st->t_factor = now_s() - t0;

    prob P = {n, rp, ci, v, Lrp, Lci, Lv, malloc(sizeof(double) * (size_t)n)};
    size_t N = (size_t)n;
    double *Qm = malloc(sizeof(double) * N * (p + 1)); /* rows: v_1..v_{j-1}, u */
    double *Au = malloc(sizeof(double) * N), *r = malloc(sizeof(double) * N), *s = malloc(sizeof(double) * N);
    double *work = malloc(sizeof(double) * N * 9);
    double *xn = malloc(sizeof(double) * N);
    double *yk = malloc(sizeof(double) * N);
    pairs_t W = {0, o->kmax, n, malloc(sizeof(double) * N * (o->kmax > 0 ? o->kmax : 1)),
                 malloc(sizeof(double) * N * (o->kmax > 0 ? o->kmax : 1)), {0}};
    double lam[OR_MAXP];
    double z[OR_MAXP + 1];
    int allconv = 1;

    if (o->jd && (o->jd_mmin < 1 || o->jd_mmax <= o->jd_mmin || o->jd_mmax > 60)) return -1;
    for (int j = 0; j < p; j++) {
        double *u = Qm + (size_t)j * N; /* becomes v_{j+1} */
        if (o->jd) {
            double tn = now_s(), th, rnj;
            st->outer_its[j] = jd_pair(&P, o, j, Qm, x0 + (size_t)j * N, &W, st, &th, &rnj, work, Au, r, s, trace,
                                       trace_cap);
            st->relres[j] = rnj / th;
            st->converged[j] = (rnj <= o->tol * th);
            if (!st->converged[j]) allconv = 0;
            lam[j] = th;
            st->t_newton += now_s() - tn;
            continue;
        }
        double td = now_s();
        /* DACG to tau_DACG before Newton, or to the final tau when it runs alone */
        st->dacg_its[j] = or_dacg(&P, j, Qm, x0 + (size_t)j * N, o->newton ? o->tol_dacg : o->tol, o->itmax_dacg, u,
                                  NULL, 0, &st->mvp_dacg, work);
        st->t_dacg += now_s() - td;

        double tn = now_s();
        W.k = 0; /* history restarts with each eigenpair */
        or_spmv(n, rp, ci, v, u, Au);
        st->mvp_newton++;
        double theta = dot(n, u, Au);
        for (int i = 0; i < n; i++) r[i] = Au[i] - theta * u[i];
        double rn = nrm2(n, r);
        int k = 0, slow = 0, restarts = 0;
        double t_restart = 0.0; /* DACG time inside the Newton phase: counted in t_dacg only */
        while (o->newton && rn > o->tol * theta && k < o->itmax) {
            int its = 0;
            int why = or_pcg(&P, theta, j + 1, Qm, u, Au, r, W.k, W.S, W.R, W.alpha, o->tol_pcg, o->itmax_pcg,
                             o->tol, o->exit_rule, o->exit_xi, s, &its, work);
            if (why == PCG_EXIT_BREAKDOWN) st->pcg_breakdowns++;
            st->pcg_its[j] += its;
            st->mvp_newton += its;
            double alpha = dot(n, s, r);
            double sn2 = dot(n, s, s);
            /* u_{k+1} = (u_k + s)/||u_k + s||, eq. (3.1); re-orthogonalise against v_1..v_{j-1} */
            for (int i = 0; i < n; i++) xn[i] = u[i] + s[i];
            scal(n, 1.0 / nrm2(n, xn), xn);
            cgs(n, j, Qm, xn, z);
            cgs(n, j, Qm, xn, z);
            scal(n, 1.0 / nrm2(n, xn), xn);
            /* store the pair (s_k, r_k) (Alg. 2) unless it would break positive definiteness */
            if (!o->bfgs_full) {
                if (alpha < -1e-12 * sqrt(sn2) * rn) pairs_push(&W, s, r, alpha);
                else st->bfgs_skipped++;
            } else {
                copy(n, r, yk); /* r_k, kept for y_k once r_{k+1} is known */
            }
            copy(n, xn, u);
            or_spmv(n, rp, ci, v, u, Au);
            st->mvp_newton++;
            double theta1 = dot(n, u, Au);
            for (int i = 0; i < n; i++) r[i] = Au[i] - theta1 * u[i];
            double rn1 = nrm2(n, r);
            if (o->bfgs_full) {
                /* eq. (2.1) with y_k = r_{k+1} - r_k: the stored vector is -y_k = r_k - r_{k+1} and
                   alpha = s^T(-y_k) < 0 is the curvature condition s^T y > 0 */
                for (int i = 0; i < n; i++) yk[i] -= r[i];
                double ay = dot(n, s, yk);
                if (ay < -1e-12 * sqrt(sn2) * nrm2(n, yk)) pairs_push(&W, s, yk, ay);
                else st->bfgs_skipped++;
            }
            if (trace && st->ntrace < trace_cap) {
                double *T = trace + 8 * (size_t)st->ntrace++;
                T[0] = j; T[1] = k; T[2] = theta; T[3] = rn; T[4] = alpha; T[5] = sn2; T[6] = theta1; T[7] = its;
            }
            /* stall: no PCG step, or the residual fails to drop below 0.9x twice in a row */
            slow = (its == 0 || rn1 > 0.9 * rn) ? slow + 1 : 0;
            theta = theta1;
            rn = rn1;
            k++;
            if ((its == 0 || slow >= 2) && restarts < 5 && rn > o->tol * theta && k < o->itmax) {
                /* return to DACG from the current iterate with a tighter tolerance, restart the BFGS history */
                double t2 = 0.005 * rn / theta;
                if (t2 > o->tol_dacg) t2 = o->tol_dacg;
                if (t2 < o->tol) t2 = o->tol;
                double td2 = now_s();
                int dits = or_dacg(&P, j, Qm, u, t2, o->itmax_dacg, xn, NULL, 0, &st->mvp_dacg, work);
                st->dacg_its[j] += dits;
                td2 = now_s() - td2;
                st->t_dacg += td2;
                t_restart += td2;
                copy(n, xn, u);
                cgs(n, j, Qm, u, z);
                cgs(n, j, Qm, u, z);
                scal(n, 1.0 / nrm2(n, u), u);
                W.k = 0;
                or_spmv(n, rp, ci, v, u, Au);
                st->mvp_newton++;
                double theta0 = theta, rn0 = rn;
                theta = dot(n, u, Au);
                for (int i = 0; i < n; i++) r[i] = Au[i] - theta * u[i];
                rn = nrm2(n, r);
                if (trace && st->ntrace < trace_cap) {
                    double *T = trace + 8 * (size_t)st->ntrace++;
                    T[0] = j; T[1] = -1; T[2] = t2; T[3] = dits; T[4] = theta; T[5] = rn; T[6] = theta0; T[7] = rn0;
                }
                restarts++;
                st->dacg_restarts++;
                slow = 0;
            }
        }
        st->outer_its[j] = k;
        st->relres[j] = rn / theta;
        st->converged[j] = (rn <= o->tol * theta);
        if (!st->converged[j]) allconv = 0;
        lam[j] = theta;
        st->t_newton += now_s() - tn - t_restart;
    }

    /* sort ascending; sign: first entry above 1e-12 ||v||_inf is positive */
    int idx[OR_MAXP];
    for (int j = 0; j < p; j++) idx[j] = j;
    for (int a = 1; a < p; a++)
        for (int b = a; b > 0 && lam[idx[b]] < lam[idx[b - 1]]; b--) { int t = idx[b]; idx[b] = idx[b - 1]; idx[b - 1] = t; }
    for (int j = 0; j < p; j++) {
        const double *u = Qm + (size_t)idx[j] * N;
        double *out = evecs + (size_t)j * N;
        double vmax = 0.0;
        for (int i = 0; i < n; i++) if (fabs(u[i]) > vmax) vmax = fabs(u[i]);
        double sg = 1.0;
        for (int i = 0; i < n; i++) if (fabs(u[i]) > 1e-12 * vmax) { sg = (u[i] > 0) ? 1.0 : -1.0; break; }
        for (int i = 0; i < n; i++) out[i] = sg * u[i];
        evals[j] = lam[idx[j]];
    }
    free(P.tmp); free(Qm); free(Au); free(r); free(s); free(work); free(xn); free(yk); free(W.S); free(W.R);
    free(Lrp); free(Lci); free(Lv);
    st->status = allconv ? 0 : 1;
    return st->status;
}

/*
 * Gradient of L(lambda, V) with respect to the stored CSR values, given the
 * eigenpairs of a symmetric A (rows of evecs), g_evals = dL/dlambda and
 * g_evecs = dL/dV (p x n, may be NULL).  Standard first-order perturbation
 * theory for simple eigenvalues:
 *   dlambda_i = v_i^T dA v_i,   dv_i = -(A - lambda_i I)^+ dA v_i.
 * xi_i = (A - lambda_i I)^+ (I - v_i v_i^T) G_i is split into the explicit
 * part along v_1..v_{i-1} and eta_i, the solution in the complement of
 * [v_1..v_i] of (I-QQ^T)(A - lambda_i I)(I-QQ^T) eta = (I-QQ^T) G_i, found by
 * PCG preconditioned with (L L^T)^{-1} and projected against Q (to tol).
 *   g_vals[e=(a,b)] = sum_i g_evals_i v_i[a] v_i[b] - 1/2 sum_i (xi_i[a] v_i[b] + v_i[a] xi_i[b])
 * Returns the largest PCG iteration count used, or <0 on failure.
 */
int or_backward(int n, const int *rp, const int *ci, const double *v, int p, const double *evals,
                const double *evecs, const double *g_evals, const double *g_evecs, double tol, int itmax,
                double shift0, double shift_max, double *g_vals) {
    size_t N = (size_t)n;
    int nnz = rp[n];
    int nnzL = or_tril_nnz(n, rp, ci);
    int *Lrp = malloc(sizeof(int) * (N + 1));
    int *Lci = malloc(sizeof(int) * (size_t)nnzL);
    double *Lv = malloc(sizeof(double) * (size_t)nnzL);
    double sh;
    if (or_ic0(n, rp, ci, v, shift0, shift_max, Lrp, Lci, Lv, &sh) != 0) { free(Lrp); free(Lci); free(Lv); return -2; }
    prob P = {n, rp, ci, v, Lrp, Lci, Lv, malloc(sizeof(double) * N)};
    double *xi = malloc(sizeof(double) * N), *eta = malloc(sizeof(double) * N), *g = malloc(sizeof(double) * N);
    double *c = malloc(sizeof(double) * N), *pv = malloc(sizeof(double) * N), *y = malloc(sizeof(double) * N);
    double *pp = malloc(sizeof(double) * N), *Ap = malloc(sizeof(double) * N);
    double z[OR_MAXP + 1];
    int maxits = 0;

    for (int e = 0; e < nnz; e++) g_vals[e] = 0.0;
    for (int i = 0; i < p; i++) {
        const double *vi = evecs + (size_t)i * N;
        for (int a = 0; a < n; a++)
            for (int e = rp[a]; e < rp[a + 1]; e++) g_vals[e] += g_evals[i] * vi[a] * vi[ci[e]];
        if (!g_evecs) continue;
        const double *G = g_evecs + (size_t)i * N;
        double gn = nrm2(n, G);
        if (gn == 0.0) continue;
        /* explicit part along v_j, j < i */
        for (int a = 0; a < n; a++) xi[a] = 0.0;
        for (int j = 0; j < i; j++) {
            const double *vj = evecs + (size_t)j * N;
            axpy(n, dot(n, vj, G) / (evals[j] - evals[i]), vj, xi);
        }
        /* eta: projected PCG in the complement of Q = [v_1..v_i] */
        int m = i + 1;
        copy(n, G, g);
        cgs(n, m, evecs, g, z);
        cgs(n, m, evecs, g, z);
        double g0 = nrm2(n, g);
        for (int a = 0; a < n; a++) eta[a] = 0.0;
        int its = 0;
        if (g0 > 0.0) {
            ic_apply(&P, g, c);
            cgs(n, m, evecs, c, z);
            double rho = dot(n, g, c);
            copy(n, c, pv);
            for (its = 1; its <= itmax; its++) {
                japply(&P, evals[i], m, evecs, pv, pp, Ap, y, z);
                double pJp = dot(n, pv, y);
                if (!(pJp > 0.0)) break;
                double gamma = rho / pJp;
                axpy(n, gamma, pv, eta);
                axpy(n, -gamma, y, g);
                if (nrm2(n, g) <= tol * g0) break;
                ic_apply(&P, g, c);
                cgs(n, m, evecs, c, z);
                double rho1 = dot(n, g, c);
                double beta = rho1 / rho;
                for (int a = 0; a < n; a++) pv[a] = c[a] + beta * pv[a];
                rho = rho1;
            }
        }
        if (its > maxits) maxits = its;
        axpy(n, 1.0, eta, xi);
        for (int a = 0; a < n; a++)
            for (int e = rp[a]; e < rp[a + 1]; e++) {
                int b = ci[e];
                g_vals[e] -= 0.5 * (xi[a] * vi[b] + vi[a] * xi[b]);
            }
    }
    free(P.tmp); free(xi); free(eta); free(g); free(c); free(pv); free(y); free(pp); free(Ap);
    free(Lrp); free(Lci); free(Lv);
    return maxits;
}

/* ------------------------------------------- thin entry points for tests */
/* Alg. 1 on caller-supplied pairs and factor (for the identity tests). */
void or_bfgspk_apply(int n, const int *Lrp, const int *Lci, const double *Lv, int k, const double *S,
                     const double *R, int m, const double *Q, const double *g, double *c) {
    double *tmp = malloc(sizeof(double) * (size_t)n), *w = malloc(sizeof(double) * (size_t)n);
    double alpha[64], a[64], z[OR_MAXP + 1];
    prob P = {n, NULL, NULL, NULL, Lrp, Lci, Lv, tmp};
    for (int s = 0; s < k; s++) alpha[s] = dot(n, S + (size_t)s * n, R + (size_t)s * n);
    or_bfgspk(&P, k, S, R, alpha, m, Q, g, c, w, a, z);
    free(tmp); free(w);
}

/* One correction-equation solve (for the PCG identity tests). */
int or_pcg_apply(int n, const int *rp, const int *ci, const double *v, const int *Lrp, const int *Lci,
                 const double *Lv, double theta, int m, const double *Q, const double *u, const double *Au,
                 const double *r, int k, const double *S, const double *R, double tol_pcg, int itmax_pcg,
                 double tau, int exit_rule, double xi, double *s, int *its) {
    size_t N = (size_t)n;
    double *work = malloc(sizeof(double) * N * 9), *tmp = malloc(sizeof(double) * N);
    double alpha[64];
    prob P = {n, rp, ci, v, Lrp, Lci, Lv, tmp};
    for (int t = 0; t < k; t++) alpha[t] = dot(n, S + (size_t)t * N, R + (size_t)t * N);
    int why = or_pcg(&P, theta, m, Q, u, Au, r, k, S, R, alpha, tol_pcg, itmax_pcg, tau, exit_rule, xi, s, its, work);
    free(work); free(tmp);
    return why;
}

/* The k_max window (Sec. 4.4) after npush pairs (rows of S and R, in the order they were produced) went
 * through it, then Alg. 1 with the pairs it kept (for the window-order tests).  Returns how many it kept. */
int or_window_apply(int n, const int *Lrp, const int *Lci, const double *Lv, int kmax, int npush, const double *S,
                    const double *R, int m, const double *Q, const double *g, double *c) {
    size_t N = (size_t)n;
    double *tmp = malloc(sizeof(double) * N), *w = malloc(sizeof(double) * N);
    double a[64], z[OR_MAXP + 1];
    pairs_t W = {0, kmax, n, malloc(sizeof(double) * N * (kmax > 0 ? kmax : 1)),
                 malloc(sizeof(double) * N * (kmax > 0 ? kmax : 1)), {0}};
    prob P = {n, NULL, NULL, NULL, Lrp, Lci, Lv, tmp};
    for (int t = 0; t < npush; t++)
        pairs_push(&W, S + (size_t)t * N, R + (size_t)t * N, dot(n, S + (size_t)t * N, R + (size_t)t * N));
    or_bfgspk(&P, W.k, W.S, W.R, W.alpha, m, Q, g, c, w, a, z);
    int kept = W.k;
    free(tmp); free(w); free(W.S); free(W.R);
    return kept;
}

/* DACG alone (for the monotone-quotient test). */
int or_dacg_apply(int n, const int *rp, const int *ci, const double *v, const int *Lrp, const int *Lci,
                  const double *Lv, int m, const double *Qt, const double *x0, double tol, int itmax,
                  double *x, double *q_hist, int hist_cap) {
    size_t N = (size_t)n;
    double *work = malloc(sizeof(double) * N * 5), *tmp = malloc(sizeof(double) * N);
    prob P = {n, rp, ci, v, Lrp, Lci, Lv, tmp};
    long long mvp = 0;
    int its = or_dacg(&P, m, Qt, x0, tol, itmax, x, q_hist, hist_cap, &mvp, work);
    free(work); free(tmp);
    return its;
}
