// CPU check of the host analysis behind the LDS-staged block solve: builds the
// partition and block schedules with the library's own code (analysis.hip), then
// emulates the block solve sequentially, checking every invariant the GPU kernel
// relies on, and compares the result with plain forward / backward substitution.
//   * blocks in order; a row's dependency is a lower rank of its block or an import
//   * an import comes from an earlier block, through an export that is already published
//   * unused register slots read the block's zero slot; padding ranks are empty
//   * virtual rows have diagonal 1 and are only read with weight -1 by their chain
//   * the output map lists the block's rows by increasing index, then its virtual rows
//   * the level-compressed systems (values from their recipes, right-hand-side
//     transform) give the same solution as the factor they come from
// Usage: check_sched <case> ; prints one line per solve and "bad N"; exit status 0 iff N = 0.
#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "internal.h"

using namespace bnx;

// 3-D grid, stencil 7 or 27 points, dof unknowns per node (lexicographic, x fastest)
static void grid(int N, int dof, bool s27, Analysis &an) {
  const int n = N * N * N * dof;
  an.n = n;
  an.rp.assign(n + 1, 0);
  an.ci.clear();
  for (int z = 0; z < N; z++)
    for (int y = 0; y < N; y++)
      for (int x = 0; x < N; x++)
        for (int d = 0; d < dof; d++) {
          const int i = (x + N * y + N * N * z) * dof + d;
          std::vector<int> cols;
          for (int dz = -1; dz <= 1; dz++)
            for (int dy = -1; dy <= 1; dy++)
              for (int dx = -1; dx <= 1; dx++) {
                if (!s27 && std::abs(dx) + std::abs(dy) + std::abs(dz) > 1) continue;
                const int X = x + dx, Y = y + dy, Z = z + dz;
                if (X < 0 || Y < 0 || Z < 0 || X >= N || Y >= N || Z >= N) continue;
                for (int e = 0; e < dof; e++) cols.push_back((X + N * Y + N * N * Z) * dof + e);
              }
          std::sort(cols.begin(), cols.end());
          for (int c : cols) an.ci.push_back(c);
          an.rp[i + 1] = (int)an.ci.size();
        }
  an.nnz = (int)an.ci.size();
}

// random geometric graph in the unit square, nodes sorted by x
static void geometric(int n, double r, unsigned seed, Analysis &an) {
  std::mt19937 g(seed);
  std::uniform_real_distribution<double> U(0, 1);
  std::vector<double> X(n), Y(n);
  for (int i = 0; i < n; i++) {
    X[i] = U(g);
    Y[i] = U(g);
  }
  std::vector<int> o(n);
  for (int i = 0; i < n; i++) o[i] = i;
  std::sort(o.begin(), o.end(), [&](int a, int b) { return X[a] < X[b]; });
  std::vector<double> xs(n), ys(n);
  for (int i = 0; i < n; i++) {
    xs[i] = X[o[i]];
    ys[i] = Y[o[i]];
  }
  an.n = n;
  an.rp.assign(n + 1, 0);
  an.ci.clear();
  for (int i = 0; i < n; i++) {
    int a = i;
    while (a > 0 && xs[i] - xs[a - 1] <= r) a--;
    for (int j = a; j < n && xs[j] - xs[i] <= r; j++) {
      const double dx = xs[j] - xs[i], dy = ys[j] - ys[i];
      if (dx * dx + dy * dy <= r * r) an.ci.push_back(j);
    }
    an.rp[i + 1] = (int)an.ci.size();
  }
  an.nnz = (int)an.ci.size();
}

static int bad = 0;
#define CHECK(c, msg)                          \
  do {                                         \
    if (!(c)) {                                \
      if (bad < 20) printf("  FAIL: %s\n", msg); \
      bad++;                                   \
    }                                          \
  } while (0)

// emulate one direction of the block solve; F: values of the system (valmap / diagmap positions),
// b: its right-hand side, ref: the exact solution
static double emulate(const Analysis &sys, bool lower, const std::vector<int> &rows, const std::vector<int> &pstart,
                      bool split, int nr, int cap, const std::vector<double> &F, const std::vector<double> &b,
                      const std::vector<double> &ref) {
  const int n = sys.n;
  BlockSched bs;
  block_schedule(sys, lower, rows, pstart, bs, split, nr);
  CHECK(bs.nr == nr, "slot count");
  std::vector<double> x(n, NAN), xe(std::max(bs.nexp, 1), NAN), xo(n, NAN);
  std::vector<char> done(n, 0);
  std::vector<int> blkof(n, -1);
  for (int blk = 0; blk < bs.nblocks; blk++)
    for (int k = bs.bptr[blk]; k < bs.bptr[blk] + bs.brows[blk]; k++)
      if (bs.perm[k] >= 0) blkof[bs.perm[k]] = blk;
  for (int blk = 0; blk < bs.nblocks; blk++) {
    const int nrow = bs.brows[blk], nimp = bs.iptr[blk + 1] - bs.iptr[blk];
    CHECK(nrow + nimp + 1 <= cap, "block exceeds its LDS target");
    std::vector<double> xs(nrow + nimp, NAN);
    std::vector<char> ok(nrow + nimp, 0);
    for (int e = 0; e < nimp; e++) {
      const int j = bs.irow[bs.iptr[blk] + e], src = bs.isrc[bs.iptr[blk] + e];
      CHECK(src >= 0 && src < bs.nexp && !std::isnan(xe[src]), "import of an unpublished export");
      CHECK(done[j] && blkof[j] < blk, "import from a later block");
      if (src >= 0 && src < bs.nexp) xs[nrow + e] = xe[src];
      ok[nrow + e] = 1;
    }
    int nreal = 0;
    for (int k = bs.bptr[blk]; k < bs.bptr[blk + 1]; k++) {
      const int t = k - bs.bptr[blk];
      if (t >= nrow) {
        CHECK((bs.cnt[k] & ~kLongSlice) == 0 && bs.perm[k] == -1, "padding rank not empty");
        continue;
      }
      const int sl = k / 64, lane = k % 64, row = bs.perm[k];
      nreal += row >= 0;
      CHECK(row >= 0 || bs.diagmap[k] == -1, "virtual row with a diagonal");
      double s = row >= 0 ? b[row] : 0.0;
      const double d = bs.diagmap[k] >= 0 ? F[bs.diagmap[k]] : 1.0;
      const int cnt = bs.cnt[k] & ~kLongSlice;
      for (int e = 0; e < cnt; e++) {
        int r, vm;
        if (e < nr) {
          r = bs.ref4[(size_t)e * bs.npad + k];
          vm = bs.valmap4[(size_t)e * bs.npad + k];
        } else {
          const int at = bs.slice_ptr[sl] + 64 * (e - nr) + lane;
          CHECK(at < bs.ell, "ELL entry out of range");
          if (at >= bs.ell) break;
          r = bs.ref[at];
          vm = bs.valmap[at];
        }
        CHECK(r != INT_MIN && r < 0 && vm >= -2 && vm != -1, "malformed dependency");
        const int slot = -r - 1;
        const bool ready = slot < nrow + nimp && ok[slot] && !(slot < nrow && slot >= t);
        CHECK(ready, "dependency not ready");
        if (!ready) break;
        CHECK(vm != -2 || (slot < nrow && bs.perm[bs.bptr[blk] + slot] == -1), "partial sum read from a row");
        s -= (vm >= 0 ? F[vm] : -1.0) * xs[slot];
      }
      for (int e = cnt; e < nr; e++) CHECK(bs.ref4[(size_t)e * bs.npad + k] == -(nrow + nimp) - 1, "unused slot");
      xs[t] = s / d;
      ok[t] = 1;
      if (row >= 0) {
        x[row] = s / d;
        done[row] = 1;
      }
    }
    CHECK(nreal == bs.nreal[blk], "row count");
    for (int e = bs.eptr[blk]; e < bs.eptr[blk + 1]; e++) {
      const int t = bs.erank[e];
      CHECK(t >= 0 && t < nrow && bs.perm[bs.bptr[blk] + t] >= 0, "export of a non-row");
      if (t >= 0 && t < nrow) xe[e] = xs[t];
    }
    for (int t = 0; t < nrow; t++) {
      const int r = bs.orow[bs.bptr[blk] + t], q = bs.oslot[bs.bptr[blk] + t];
      if (t < nreal) {
        CHECK(t == 0 || r > bs.orow[bs.bptr[blk] + t - 1], "output rows not increasing");
        CHECK(bs.perm[bs.bptr[blk] + q] == r, "output slot");
        xo[r] = xs[q];
      } else {
        CHECK(r == -1, "virtual row in the output");
      }
    }
  }
  double err = 0, scale = 0;
  for (int i = 0; i < n; i++) {
    err = std::max(err, std::fabs(xo[i] - ref[i]));
    scale = std::max(scale, std::fabs(ref[i]));
  }
  return err / scale;
}

static void run(Analysis &an, int cap, const char *name, bool split, bool lps, int nr_force = 0) {
  analyse(an);
  const int n = an.n;
  // a well-conditioned lower-triangular factor on the pattern (diagonal dominant)
  std::vector<double> Lv(an.nnzL), Ltv(an.nnzL), b(n);
  for (int i = 0; i < n; i++)
    for (int q = an.Lrp[i]; q < an.Lrp[i + 1]; q++)
      Lv[q] = (q == an.Lrp[i + 1] - 1) ? 3.0 + (i % 7) * 0.1 : -0.3 - (q % 5) * 0.05;
  for (int q = 0; q < an.nnzL; q++) Ltv[q] = Lv[an.mapLt[q]];
  for (int i = 0; i < n; i++) b[i] = std::sin(0.37 * i) + 0.1;
  std::vector<double> ref[2] = {std::vector<double>(n), std::vector<double>(n)};
  for (int i = 0; i < n; i++) {
    double s = b[i];
    for (int q = an.Lrp[i]; q < an.Lrp[i + 1] - 1; q++) s -= Lv[q] * ref[0][an.Lci[q]];
    ref[0][i] = s / Lv[an.Lrp[i + 1] - 1];
  }
  for (int i = n - 1; i >= 0; i--) {
    double s = b[i];
    for (int q = an.Ltrp[i] + 1; q < an.Ltrp[i + 1]; q++) s -= Ltv[q] * ref[1][an.Ltci[q]];
    ref[1][i] = s / Ltv[an.Ltrp[i]];
  }
  Analysis cs;
  std::vector<double> F[2] = {Lv, Ltv}, rhs[2] = {b, b};
  const Analysis *sys = &an;
  int nr = kNR;
  if (lps) {
    SolveSys Sf, Sb;
    const bool ok = compress_both(an, split, Sf, Sb);
    printf("%s: level-pair substitution %s (levels %d -> %d, %d -> %d, entries %d -> %d)\n", name,
           ok ? "applies" : "rejected", an.levL.nlev, Sf.nlev, an.levLt.nlev, Sb.nlev, an.nnzL, Sf.nnz);
    if (!ok) return;
    // the counting pass that screens a substitution counts exactly the entries the build writes
    for (int d = 0; d < 2; d++) {
      const SolveSys &S = d == 0 ? Sf : Sb;
      SolveSys T;
      CHECK(compress_system(an, d == 0, INT_MAX, T, S.nnz) && T.nnz == S.nnz, "entry count admits the system");
      CHECK(!compress_system(an, d == 0, INT_MAX, T, S.nnz - 1), "entry count one short rejects it");
    }
    cs.n = n;
    cs.Lrp = Sf.rp;
    cs.Lci = Sf.ci;
    cs.Ltrp = Sb.rp;
    cs.Ltci = Sb.ci;
    cs.nnzL = Sf.nnz;
    levels_from(n, Sf.level, cs.levL);
    levels_from(n, Sb.level, cs.levLt);
    for (int d = 0; d < 2; d++) {
      const SolveSys &S = d == 0 ? Sf : Sb;
      const std::vector<double> &v = d == 0 ? Lv : Ltv;
      F[d].assign(S.nnz, 0.0);
      for (int e = 0; e < S.nnz; e++) {
        double x = S.direct[e] >= 0 ? v[S.direct[e]] : 0.0;
        for (int t = S.tp[e]; t < S.tp[e + 1]; t++) x -= v[S.ta[t]] * v[S.tb[t]] / v[S.tc[t]];
        F[d][e] = x;
      }
      for (int i = 0; i < n; i++) {
        double x = b[i];
        for (int t = S.mp[i]; t < S.mp[i + 1]; t++) x -= v[S.ma[t]] / v[S.mc[t]] * b[S.mj[t]];
        rhs[d][i] = x;
      }
      // levels strictly increase along every dependency of the compressed system
      for (int i = 0; i < n; i++) {
        const int a = d == 0 ? S.rp[i] : S.rp[i] + 1, z = d == 0 ? S.rp[i + 1] - 1 : S.rp[i + 1];
        CHECK(split || z - a <= kNRC, "compressed row longer than kNRC");
        for (int e = a; e < z; e++) CHECK(S.level[S.ci[e]] < S.level[i], "compressed level order");
      }
    }
    sys = &cs;
  }
  nr = nr_force ? nr_force : slots_for(*sys, lps);
  std::vector<int> rows, pstart;
  if (!partition_rows(*sys, cap, rows, pstart, split, nr, lps ? &an : nullptr)) {
    printf("%s: partition infeasible\n", name);
    bad++;
    return;
  }
  for (int d = 0; d < 2; d++) {
    const double err = emulate(*sys, d == 0, rows, pstart, split, nr, cap, F[d], rhs[d], ref[d]);
    printf("%s%s%s %s: blocks %zu, slots %d, error %.2e\n", name, split ? " split" : "", lps ? " lps" : "",
           d == 0 ? "forward" : "backward", pstart.size() - 1, nr, err);
    CHECK(err < 1e-10, "solution differs from substitution");
  }
}

int main(int argc, char **argv) {
  const char *c = argc > 1 ? argv[1] : "all";
  auto want = [&](const char *k) { return !strcmp(c, "all") || !strcmp(c, k); };
  for (int v = 0; v < 3; v++) {  // plain, split, split + level-pair substitution
    const bool split = v > 0, lps = v == 2;
    if (want("grid")) {
      Analysis a;
      grid(24, 1, false, a);
      run(a, 2048, "7-point 24^3", split, lps);
      Analysis b;
      grid(13, 1, false, b);
      run(b, 512, "7-point 13^3 (small blocks)", split, lps);
    }
    if (want("elasticity")) {
      Analysis a;
      grid(8, 3, true, a);
      run(a, 900, "27-point 8^3 x 3 dof", split, lps);
      if (split && !lps)  // the other slot counts of split schedules
        for (int nrf : {kNRC, kNRW}) {
          Analysis b;
          grid(8, 3, true, b);
          run(b, 900, "27-point 8^3 x 3 dof", split, lps, nrf);
        }
    }
    if (want("graph")) {
      Analysis a;
      geometric(4000, 0.03, 3, a);
      run(a, 900, "geometric graph 4000", split, lps);
      if (split && !lps)
        for (int nrf : {kNRC, kNRW}) {
          Analysis b;
          geometric(4000, 0.03, 3, b);
          run(b, 900, "geometric graph 4000", split, lps, nrf);
        }
    }
  }
  printf("bad %d\n", bad);
  return bad != 0;
}
