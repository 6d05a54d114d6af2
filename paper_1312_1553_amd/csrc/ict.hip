// IC(lfil, tau_IC): the incomplete Cholesky factor the paper uses as its initial
// preconditioner (Sec. 2, defaults lfil = 30, tau_IC = 1e-2 in Table 2), on the
// host.  The pattern of a threshold factor depends on the values row by row, so
// it has no level structure to run in parallel; the paper computes it on the
// CPU as well.  What the GPU consumes -- the factor in CSR, its transpose, level
// sets and the LDS block schedules of the two triangular solves -- is built from
// the result exactly as for IC(0).
//
// The paper names only the two parameters.  The dual dropping rule (ILUT style):
//  * the factor Ls is computed for As = D^-1/2 A D^-1/2 (D = diag(A); entry
//    (a_ij r_i) r_j with r_i = 1/sqrt(a_ii), diagonal included), so the rule does
//    not depend on the scaling of A, and L = D^1/2 Ls is returned;
//  * row i: tau_i = tau_IC ||As(i,:)||_2 (squares summed in column order);
//    w = strictly lower part of As(i,:); for k ascending over the nonzeros of w,
//    fill included: l = w_k / Ls_kk; |l| < tau_i drops the entry (it takes no part
//    in the elimination), otherwise l is a candidate and w_m -= l Ls_mk for each
//    earlier row m > k with an entry in column k (which may create fill at m);
//  * the lfil candidates largest in magnitude are kept (ties to the smaller
//    column) and Ls_ii = sqrt(As_ii - sum of their squares in column order).
// A shift a factors A + a diag(A) from scratch (scaling and thresholds included).
#include <algorithm>
#include <cmath>
#include <functional>

#include "internal.h"

namespace bnx {

bool ict_factor(int n, const int *rp, const int *ci, const double *val, int lfil, double tau, double shift,
                IctFactor &L) {
  std::vector<double> sq(n), r(n), ds(n), ti(n);
  for (int i = 0; i < n; i++) {
    double dv = 0.0;
    for (int e = rp[i]; e < rp[i + 1]; e++)
      if (ci[e] == i) dv = val[e];
    const double d = dv * (1.0 + shift);
    sq[i] = std::sqrt(d);
    r[i] = 1.0 / sq[i];
    ds[i] = d * r[i] * r[i];
  }
  for (int i = 0; i < n; i++) {
    double s2 = 0.0;
    for (int e = rp[i]; e < rp[i + 1]; e++) {
      const double as = ci[e] == i ? ds[i] : val[e] * r[i] * r[ci[e]];
      s2 += as * as;
    }
    ti[i] = tau * std::sqrt(s2);
  }
  L.rp.assign(n + 1, 0);
  L.ci.clear();
  L.v.clear();
  const size_t guess = (size_t)rp[n] + (size_t)n;
  L.ci.reserve(guess);
  L.v.reserve(guess);
  std::vector<int> rowof, nxt;  // row of each entry; next entry of the same column
  rowof.reserve(guess);
  nxt.reserve(guess);
  std::vector<int> head(n, -1), tail(n, -1), mark(n, -1);
  std::vector<double> w(n, 0.0);
  std::vector<int> heap;  // pending positions of the current row (min-heap)
  struct Cand {
    int col;
    double v;
  };
  std::vector<Cand> cand;
  for (int i = 0; i < n; i++) {
    heap.clear();
    for (int e = rp[i]; e < rp[i + 1]; e++) {
      const int j = ci[e];
      if (j >= i) break;  // columns ascend
      w[j] = val[e] * r[i] * r[j];
      mark[j] = i;
      heap.push_back(j);  // ascending, hence already a min-heap
    }
    cand.clear();
    while (!heap.empty()) {
      std::pop_heap(heap.begin(), heap.end(), std::greater<int>());
      const int k = heap.back();
      heap.pop_back();
      const double l = w[k] / L.v[L.rp[k + 1] - 1];
      w[k] = 0.0;
      mark[k] = -1;
      if (std::fabs(l) < ti[i]) continue;
      cand.push_back({k, l});
      for (int e = head[k]; e >= 0; e = nxt[e]) {
        const int m = rowof[e];
        if (mark[m] != i) {
          mark[m] = i;
          heap.push_back(m);
          std::push_heap(heap.begin(), heap.end(), std::greater<int>());
        }
        w[m] -= l * L.v[e];
      }
    }
    if ((int)cand.size() > lfil) {
      std::sort(cand.begin(), cand.end(), [](const Cand &a, const Cand &b) {
        const double x = std::fabs(a.v), y = std::fabs(b.v);
        return x != y ? x > y : a.col < b.col;
      });
      cand.resize(lfil);
      std::sort(cand.begin(), cand.end(), [](const Cand &a, const Cand &b) { return a.col < b.col; });
    }
    double d = ds[i];
    for (const Cand &c : cand) d -= c.v * c.v;
    if (!(d > 0.0)) return false;
    for (const Cand &c : cand) {
      const int e = (int)L.v.size();
      L.ci.push_back(c.col);
      L.v.push_back(c.v);
      rowof.push_back(i);
      nxt.push_back(-1);
      if (tail[c.col] < 0) head[c.col] = e;
      else nxt[tail[c.col]] = e;
      tail[c.col] = e;
    }
    L.ci.push_back(i);
    L.v.push_back(std::sqrt(d));
    rowof.push_back(i);
    nxt.push_back(-1);
    L.rp[i + 1] = (int)L.v.size();
    if ((long long)L.v.size() > (long long)INT32_MAX - n) return false;
  }
  for (int i = 0; i < n; i++)
    for (int e = L.rp[i]; e < L.rp[i + 1]; e++) L.v[e] *= sq[i];
  return true;
}

void pattern_of_factor(int n, const IctFactor &L, Analysis &an) {
  // symmetric pattern L + L^T in CSR with ascending columns: row j holds the
  // entries of row j of L (diagonal last), then (j, i) for L(i, j) != 0, i ascending
  an = Analysis{};
  an.n = n;
  std::vector<int> cnt(n, 0);
  for (int i = 0; i < n; i++) {
    cnt[i] += L.rp[i + 1] - L.rp[i];
    for (int e = L.rp[i]; e < L.rp[i + 1] - 1; e++) cnt[L.ci[e]]++;
  }
  an.rp.assign(n + 1, 0);
  for (int i = 0; i < n; i++) an.rp[i + 1] = an.rp[i] + cnt[i];
  an.nnz = an.rp[n];
  an.ci.resize(an.nnz);
  std::vector<int> fill(n);
  for (int i = 0; i < n; i++) {
    fill[i] = an.rp[i];
    for (int e = L.rp[i]; e < L.rp[i + 1]; e++) an.ci[fill[i]++] = L.ci[e];
  }
  for (int i = 0; i < n; i++)
    for (int e = L.rp[i]; e < L.rp[i + 1] - 1; e++) an.ci[fill[L.ci[e]]++] = i;
}

}  // namespace bnx
