// Host-side analysis of the CSR pattern: validation, IC(0) pattern of tril(A),
// the transposed factor pattern and the level schedules of both triangular
// solves.  Index work only; the factorisation itself runs on the device.
#include <algorithm>
#include <cstdio>

#include "internal.h"

namespace bnx {

std::string validate_csr(int n, int nnz, const int *rp, const int *ci) {
  char buf[256];
  if (n < 1) return "n must be >= 1";
  if (rp[0] != 0) return "rowptr[0] must be 0";
  if (rp[n] != nnz) return "rowptr[n] must equal nnz";
  for (int i = 0; i < n; i++) {
    if (rp[i + 1] < rp[i]) {
      snprintf(buf, sizeof buf, "rowptr decreases at row %d", i);
      return buf;
    }
    bool diag = false;
    for (int e = rp[i]; e < rp[i + 1]; e++) {
      int j = ci[e];
      if (j < 0 || j >= n) {
        snprintf(buf, sizeof buf, "column %d out of range in row %d", j, i);
        return buf;
      }
      if (e > rp[i] && ci[e - 1] >= j) {
        snprintf(buf, sizeof buf, "columns not strictly increasing in row %d", i);
        return buf;
      }
      diag |= (j == i);
    }
    if (!diag) {
      snprintf(buf, sizeof buf, "missing diagonal in row %d", i);
      return buf;
    }
  }
  // symmetric pattern: count of (i,j) must match (j,i)
  std::vector<int> cnt(n, 0);
  for (int e = 0; e < nnz; e++) cnt[ci[e]]++;
  for (int i = 0; i < n; i++)
    if (cnt[i] != rp[i + 1] - rp[i]) {
      snprintf(buf, sizeof buf, "pattern not symmetric (row/column %d)", i);
      return buf;
    }
  std::vector<int> pos(rp, rp + n);  // fill pointer per column
  // every (i,j) must have (j,i): scan rows in order; columns of the transpose fill in row order
  std::vector<int> tci(nnz);
  for (int i = 0; i < n; i++)
    for (int e = rp[i]; e < rp[i + 1]; e++) tci[pos[ci[e]]++] = i;
  for (int e = 0; e < nnz; e++)
    if (tci[e] != ci[e]) return "pattern not symmetric";
  return "";
}

static void build_levels(int n, const std::vector<int> &lev, Levels &L) {
  L.level = lev;
  int nlev = 0;
  for (int i = 0; i < n; i++) nlev = std::max(nlev, lev[i] + 1);
  L.nlev = nlev;
  L.ptr.assign(nlev + 1, 0);
  for (int i = 0; i < n; i++) L.ptr[lev[i] + 1]++;
  for (int l = 0; l < nlev; l++) L.ptr[l + 1] += L.ptr[l];
  std::vector<int> fill(L.ptr.begin(), L.ptr.end() - 1);
  L.rows.assign(n, 0);
  for (int i = 0; i < n; i++) L.rows[fill[lev[i]]++] = i;
  L.max_rows = 0;
  for (int l = 0; l < nlev; l++) L.max_rows = std::max(L.max_rows, L.ptr[l + 1] - L.ptr[l]);
}

void analyse(Analysis &an) {
  const int n = an.n;
  const auto &rp = an.rp, &ci = an.ci;
  // L = pattern of tril(A), rows keep A's column order (diagonal last)
  an.Lrp.assign(n + 1, 0);
  for (int i = 0; i < n; i++) {
    int c = 0;
    for (int e = rp[i]; e < rp[i + 1]; e++) c += (ci[e] <= i);
    an.Lrp[i + 1] = an.Lrp[i] + c;
  }
  an.nnzL = an.Lrp[n];
  an.Lci.resize(an.nnzL);
  an.mapL.resize(an.nnzL);
  for (int i = 0; i < n; i++) {
    int c = an.Lrp[i];
    for (int e = rp[i]; e < rp[i + 1]; e++)
      if (ci[e] <= i) {
        an.Lci[c] = ci[e];
        an.mapL[c] = e;
        c++;
      }
  }
  // L^T in CSR: row j holds (j, i) for L(i, j) != 0, i ascending -> diagonal first
  an.Ltrp.assign(n + 1, 0);
  for (int q = 0; q < an.nnzL; q++) an.Ltrp[an.Lci[q] + 1]++;
  for (int j = 0; j < n; j++) an.Ltrp[j + 1] += an.Ltrp[j];
  an.Ltci.resize(an.nnzL);
  an.mapLt.resize(an.nnzL);
  std::vector<int> fill(an.Ltrp.begin(), an.Ltrp.end() - 1);
  for (int i = 0; i < n; i++)
    for (int q = an.Lrp[i]; q < an.Lrp[i + 1]; q++) {
      int j = an.Lci[q];
      an.Ltci[fill[j]] = i;
      an.mapLt[fill[j]] = q;
      fill[j]++;
    }
  // levels of the forward solve: lev(i) = 1 + max lev(j), j < i in row i of L
  std::vector<int> lev(n, 0);
  for (int i = 0; i < n; i++) {
    int l = 0;
    for (int q = an.Lrp[i]; q < an.Lrp[i + 1] - 1; q++) l = std::max(l, lev[an.Lci[q]] + 1);
    lev[i] = l;
  }
  build_levels(n, lev, an.levL);
  // levels of the backward solve: row i of L^T depends on j > i
  for (int i = n - 1; i >= 0; i--) {
    int l = 0;
    for (int q = an.Ltrp[i] + 1; q < an.Ltrp[i + 1]; q++) l = std::max(l, lev[an.Ltci[q]] + 1);
    lev[i] = l;
  }
  build_levels(n, lev, an.levLt);
}

void block_schedule(const Analysis &an, bool lower, int B, BlockSched &bs) {
  const int n = an.n;
  const std::vector<int> &rp = lower ? an.Lrp : an.Ltrp;
  const std::vector<int> &ci = lower ? an.Lci : an.Ltci;
  bs.n = n;
  bs.B = B;
  bs.nblocks = (n + B - 1) / B;
  auto pos_of = [&](int i) { return lower ? i : n - 1 - i; };
  auto row_at = [&](int p) { return lower ? p : n - 1 - p; };
  // sort key: level of the row in the whole dependency graph
  const std::vector<int> &glev = lower ? an.levL.level : an.levLt.level;
  std::vector<int> llev(n, 0);
  bs.max_local_levels = 0;
  for (int p = 0; p < n; p++) {
    llev[p] = glev[row_at(p)];
  }
  for (int b = 0; b < bs.nblocks; b++) {
    int lo = INT32_MAX, hi = -1;
    for (int p = b * B; p < std::min(n, b * B + B); p++) {
      lo = std::min(lo, llev[p]);
      hi = std::max(hi, llev[p]);
    }
    bs.max_local_levels = std::max(bs.max_local_levels, hi - lo + 1);
  }
  // sort each block by (level, position)
  bs.perm.assign(n, 0);
  bs.diagmap.assign(n, 0);
  std::vector<int> rank(n, 0), order;
  for (int b = 0; b < bs.nblocks; b++) {
    const int p0 = b * B, p1 = std::min(n, p0 + B);
    order.resize(p1 - p0);
    for (int p = p0; p < p1; p++) order[p - p0] = p;
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return llev[a] < llev[c]; });
    for (int k = p0; k < p1; k++) {
      const int i = row_at(order[k - p0]);
      bs.perm[k] = i;
      rank[i] = k;
      bs.diagmap[k] = lower ? rp[i + 1] - 1 : rp[i];
    }
  }
  // first kNR dependencies per rank, rank-indexed
  bs.cnt.assign(n, 0);
  bs.ref4.assign((size_t)kNR * n, INT32_MIN);
  bs.valmap4.assign((size_t)kNR * n, -1);
  // ELL slices of 64 ranks for the dependencies beyond kNR
  bs.nslices = (n + 63) / 64;
  bs.slice_ptr.assign(bs.nslices + 1, 0);
  bs.slice_nnz.assign(bs.nslices, 0);
  for (int sl = 0; sl < bs.nslices; sl++) {
    int mx = 0;
    for (int k = sl * 64; k < std::min(n, sl * 64 + 64); k++) {
      const int i = bs.perm[k];
      mx = std::max(mx, rp[i + 1] - rp[i] - 1 - kNR);
    }
    bs.slice_nnz[sl] = mx;
    bs.slice_ptr[sl + 1] = bs.slice_ptr[sl] + 64 * mx;
  }
  bs.ell = bs.slice_ptr[bs.nslices];
  bs.ref.assign(bs.ell, INT32_MIN);
  bs.valmap.assign(bs.ell, -1);
  for (int k = 0; k < n; k++) {
    const int sl = k / 64, lane = k % 64;
    const int i = bs.perm[k];
    const int b0 = (k / B) * B;  // first rank of the block
    const int e0 = lower ? rp[i] : rp[i] + 1, e1 = lower ? rp[i + 1] - 1 : rp[i + 1];
    bs.cnt[k] = e1 - e0;
    int e = 0;
    for (int q = e0; q < e1; q++, e++) {
      const int kj = rank[ci[q]];
      const int r = (kj >= b0) ? -(kj - b0) - 1 : kj;
      if (e < kNR) {
        bs.ref4[(size_t)e * n + k] = r;
        bs.valmap4[(size_t)e * n + k] = q;
      } else {
        const int at = bs.slice_ptr[sl] + 64 * (e - kNR) + lane;
        bs.ref[at] = r;
        bs.valmap[at] = q;
      }
    }
  }
}

}  // namespace bnx
