// Host-side analysis of the CSR pattern: validation, IC(0) pattern of tril(A),
// the transposed factor pattern and the level schedules of both triangular
// solves.  Index work only; the factorisation itself runs on the device.
#include <algorithm>
#include <array>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>

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

void levels_from(int n, const std::vector<int> &lev, Levels &L) { build_levels(n, lev, L); }

int slots_for(const Analysis &sys, bool compressed) {
  int m = 0;
  for (int i = 0; i < sys.n; i++)
    m = std::max(m, std::max(sys.Lrp[i + 1] - sys.Lrp[i], sys.Ltrp[i + 1] - sys.Ltrp[i]) - 1);
  if (m <= 3) return 3;
  return compressed ? kNRC : kNR;
}

bool compress_system(const Analysis &an, bool lower, int maxdeps, SolveSys &S, long long max_entries) {
  const int n = an.n;
  const std::vector<int> &rp = lower ? an.Lrp : an.Ltrp;
  const std::vector<int> &ci = lower ? an.Lci : an.Ltci;
  const std::vector<int> &lev = lower ? an.levL.level : an.levLt.level;
  const int nlev0 = lower ? an.levL.nlev : an.levLt.nlev;
  auto deps = [&](int i, int &e0, int &e1) {
    e0 = lower ? rp[i] : rp[i] + 1;
    e1 = lower ? rp[i + 1] - 1 : rp[i + 1];
  };
  auto diag = [&](int i) { return lower ? rp[i + 1] - 1 : rp[i]; };
  S = SolveSys{};
  {
    // counting pass (no recipes): reject early when a row exceeds maxdeps or the entries exceed
    // max_entries, before the recipes of a system that would be discarded are built
    std::vector<int> mark(n, -1);
    long long entries = 0;
    for (int i = 0; i < n; i++) {
      int e0, e1, cnt = 0;
      deps(i, e0, e1);
      const bool even = (lev[i] & 1) == 0;
      auto add = [&](int k) {
        if (mark[k] != i) {
          mark[k] = i;
          cnt++;
        }
      };
      for (int e = e0; e < e1; e++) {
        const int j = ci[e];
        if (even && (lev[j] & 1) == 1) {
          int f0, f1;
          deps(j, f0, f1);
          for (int f = f0; f < f1; f++) add(ci[f]);
        } else {
          add(j);
        }
      }
      entries += cnt + 1;
      if (cnt > maxdeps || entries > max_entries) return false;
    }
  }
  S.n = n;
  S.rp.assign(n + 1, 0);
  S.mp.assign(n + 1, 0);
  std::vector<int> slot(n, -1), cols;
  std::vector<int> dir;                            // direct position of each new column
  std::vector<std::vector<std::array<int, 3>>> tr;  // substitution terms of each new column
  auto push_row = [&](int i) {
    // columns ascending; the diagonal last (forward) or first (backward)
    std::vector<int> ord(cols.size());
    for (size_t t = 0; t < cols.size(); t++) ord[t] = (int)t;
    std::sort(ord.begin(), ord.end(), [&](int a, int b) { return cols[a] < cols[b]; });
    auto put = [&](int col, int d, const std::vector<std::array<int, 3>> *terms) {
      S.ci.push_back(col);
      S.direct.push_back(d);
      S.tp.push_back((int)S.ta.size());
      if (terms)
        for (const auto &x : *terms) {
          S.ta.push_back(x[0]);
          S.tb.push_back(x[1]);
          S.tc.push_back(x[2]);
        }
    };
    if (!lower) put(i, diag(i), nullptr);
    for (int t : ord) put(cols[t], dir[t], &tr[t]);
    if (lower) put(i, diag(i), nullptr);
    S.rp[i + 1] = (int)S.ci.size();
    for (int c : cols) slot[c] = -1;
  };
  bool fits = true;
  for (int i = 0; i < n; i++) {
    cols.clear();
    dir.clear();
    tr.clear();
    auto col_of = [&](int k) {
      if (slot[k] < 0) {
        slot[k] = (int)cols.size();
        cols.push_back(k);
        dir.push_back(-1);
        tr.emplace_back();
      }
      return slot[k];
    };
    int e0, e1;
    deps(i, e0, e1);
    const bool even = (lev[i] & 1) == 0;
    for (int e = e0; e < e1; e++) {
      const int j = ci[e];
      if (even && (lev[j] & 1) == 1) {  // x_j = (b_j - sum_k v_jk x_k) / v_jj substituted into row i
        S.mj.push_back(j);
        S.ma.push_back(e);
        S.mc.push_back(diag(j));
        int f0, f1;
        deps(j, f0, f1);
        for (int f = f0; f < f1; f++) tr[col_of(ci[f])].push_back({e, f, diag(j)});
      } else {
        dir[col_of(j)] = e;
      }
    }
    S.mp[i + 1] = (int)S.mj.size();
    if ((int)cols.size() > maxdeps) fits = false;
    push_row(i);
  }
  S.tp.push_back((int)S.ta.size());
  S.nnz = (int)S.ci.size();
  // levels of the new system
  S.level.assign(n, 0);
  auto level_of = [&](int i) {
    int l = 0;
    const int a = lower ? S.rp[i] : S.rp[i] + 1, b = lower ? S.rp[i + 1] - 1 : S.rp[i + 1];
    for (int e = a; e < b; e++) l = std::max(l, S.level[S.ci[e]] + 1);
    S.level[i] = l;
  };
  if (lower)
    for (int i = 0; i < n; i++) level_of(i);
  else
    for (int i = n - 1; i >= 0; i--) level_of(i);
  S.nlev = 0;
  for (int i = 0; i < n; i++) S.nlev = std::max(S.nlev, S.level[i] + 1);
  return fits && 4 * S.nlev <= 3 * nlev0;
}

bool compress_both(const Analysis &an, bool split, SolveSys &Sf, SolveSys &Sb) {
  if (compress_system(an, true, kNRC, Sf) && compress_system(an, false, kNRC, Sb)) return true;
  if (!split) return false;
  // rows beyond kNRC dependencies run as chains of virtual rows; the substitution must still
  // halve the levels without growing the entries much (on 27-point elasticity blocks it grows
  // them 2.5x and the chains lengthen the critical path instead)
  const long long cap = (3LL * an.nnzL) / 2;
  return compress_system(an, true, INT_MAX, Sf, cap) && compress_system(an, false, INT_MAX, Sb, cap);
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

// Coordinates that never decrease along a dependency of the forward solve.  The
// strictly lower entries (i, j) of L are classed by their index distance i - j:
// up to three classes, cut at the two widest gaps (at least a factor 4) between
// the frequent distances on a log scale.  Coordinate c of row i is the largest
// number of class-c steps on a dependency path ending at i.  On a grid numbered
// lexicographically these are the grid coordinates.
static int dag_coords(const Analysis &an, std::vector<int> co[3]) {
  const int n = an.n;
  std::vector<int> dist;
  dist.reserve(an.nnzL - n);
  for (int i = 0; i < n; i++)
    for (int q = an.Lrp[i]; q < an.Lrp[i + 1] - 1; q++) dist.push_back(i - an.Lci[q]);
  std::sort(dist.begin(), dist.end());
  std::vector<double> lg;  // log2 of the distances carrying at least 1 % of the entries
  const size_t m = dist.size();
  for (size_t a = 0; a < m;) {
    size_t b = a;
    while (b < m && dist[b] == dist[a]) b++;
    if ((b - a) * 100 >= m) lg.push_back(std::log2((double)dist[a]));
    a = b;
  }
  std::vector<std::pair<double, double>> gaps;  // (width, cut point)
  for (size_t t = 1; t < lg.size(); t++)
    if (lg[t] - lg[t - 1] >= 2.0) gaps.push_back({lg[t] - lg[t - 1], 0.5 * (lg[t] + lg[t - 1])});
  std::sort(gaps.rbegin(), gaps.rend());
  std::vector<double> cuts;
  for (size_t t = 0; t < gaps.size() && t < 2; t++) cuts.push_back(gaps[t].second);
  std::sort(cuts.begin(), cuts.end());
  const int ncls = (int)cuts.size() + 1;
  for (int c = 0; c < ncls; c++) co[c].assign(n, 0);
  for (int i = 0; i < n; i++)
    for (int q = an.Lrp[i]; q < an.Lrp[i + 1] - 1; q++) {
      const int j = an.Lci[q];
      const double l = std::log2((double)(i - j));
      int cls = 0;
      while (cls < (int)cuts.size() && l > cuts[cls]) cls++;
      for (int c = 0; c < ncls; c++) co[c][i] = std::max(co[c][i], co[c][j] + (c == cls));
    }
  return ncls;
}

namespace {
// Recursive bisection of the rows.  Each cut puts the rows whose value of a
// monotone coordinate is at most a threshold first; that side holds every
// predecessor (within the part) of its rows, so the leaves in depth-first
// order are a topological order of the blocks.  Among the candidate
// coordinates (the distance classes, the level, the row index) the cut with
// the fewest dependency edges across it is taken, which keeps blocks compact
// and a dependency path crosses few of them.
struct Bisect {
  const Analysis &an;
  int cap;
  std::vector<const std::vector<int> *> coord;
  std::vector<int> idx, stamp_in, stamp_l, stamp_u, side;
  int stamp = 0;
  std::vector<int> &rows, &pstart;
  bool ok = true;

  Bisect(const Analysis &a, int c, std::vector<int> &r, std::vector<int> &p) : an(a), cap(c), rows(r), pstart(p) {}
  const std::vector<int> *vl = nullptr, *vu = nullptr;  // virtual rows per row and direction (split schedules)

  bool fits(int a, int b) {
    if (b - a > cap) return false;
    ++stamp;
    for (int t = a; t < b; t++) stamp_in[rows[t]] = stamp;
    int imp_l = 0, imp_u = 0;
    long virt_l = 0, virt_u = 0;
    for (int t = a; t < b; t++) {
      const int i = rows[t];
      if (vl) {
        virt_l += (*vl)[i];
        virt_u += (*vu)[i];
      }
      for (int q = an.Lrp[i]; q < an.Lrp[i + 1] - 1; q++) {
        const int j = an.Lci[q];
        if (stamp_in[j] != stamp && stamp_l[j] != stamp) {
          stamp_l[j] = stamp;
          imp_l++;
        }
      }
      for (int q = an.Ltrp[i] + 1; q < an.Ltrp[i + 1]; q++) {
        const int j = an.Ltci[q];
        if (stamp_in[j] != stamp && stamp_u[j] != stamp) {
          stamp_u[j] = stamp;
          imp_u++;
        }
      }
    }
    return (b - a) + std::max(imp_l + virt_l, imp_u + virt_u) + 1 <= cap;  // + the zero slot
  }
  int value(int c, int i) const { return c < (int)coord.size() ? (*coord[c])[i] : i; }
  // threshold of coordinate c splitting rows[a, b) nearest to half; false if it cannot split
  bool threshold(int c, int a, int b, int &thr) {
    std::vector<int> v(b - a);
    for (int t = a; t < b; t++) v[t - a] = value(c, rows[t]);
    const int h = (b - a) / 2;
    std::nth_element(v.begin(), v.begin() + h, v.end());
    const int med = v[h];
    int below = 0, at = 0;
    for (int x : v) {
      below += x < med;
      at += x == med;
    }
    // cut after med (below + at rows first) or before it (below rows first)
    const int n1 = below + at, n0 = below;
    const bool ok1 = n1 < b - a, ok0 = n0 > 0;
    if (!ok1 && !ok0) return false;
    if (ok1 && (!ok0 || std::abs(n1 - h) <= std::abs(n0 - h))) thr = med;
    else thr = med - 1;
    return true;
  }
  long cut_edges(int c, int a, int b, int thr) {
    ++stamp;
    for (int t = a; t < b; t++) {
      stamp_in[rows[t]] = stamp;
      side[rows[t]] = value(c, rows[t]) <= thr ? 0 : 1;
    }
    long cut = 0;
    for (int t = a; t < b; t++) {
      const int i = rows[t];
      for (int q = an.Lrp[i]; q < an.Lrp[i + 1] - 1; q++) {
        const int j = an.Lci[q];
        cut += stamp_in[j] == stamp && side[j] != side[i];
      }
    }
    return cut;
  }
  void run(int a, int b) {
    if (!ok) return;
    if (fits(a, b)) {
      pstart.push_back(b);
      return;
    }
    if (b - a == 1) {  // a single row that needs more than the LDS holds
      ok = false;
      return;
    }
    int best_c = -1, best_thr = 0;
    long best_cut = -1;
    for (int c = 0; c <= (int)coord.size(); c++) {
      int thr;
      if (!threshold(c, a, b, thr)) continue;
      const long cut = cut_edges(c, a, b, thr);
      if (best_c < 0 || cut < best_cut) {
        best_c = c;
        best_cut = cut;
        best_thr = thr;
      }
    }
    // the row index always splits a part of two or more rows
    const int c = best_c, thr = best_thr;
    auto mid = std::stable_partition(rows.begin() + a, rows.begin() + b,
                                     [&](int i) { return value(c, i) <= thr; });
    const int m = (int)(mid - rows.begin());
    run(a, m);
    run(m, b);
  }
};
}  // namespace

int virtual_rows(int deps, int nr) { return deps <= nr ? 0 : (deps - nr + nr - 2) / (nr - 1); }

bool partition_rows(const Analysis &an, int cap, std::vector<int> &rows, std::vector<int> &pstart, bool split,
                    int nr, const Analysis *order) {
  const int n = an.n;
  // the coordinates that order the blocks come from `order` (default: an itself): a graph whose
  // edges, in both solve directions, compose every dependency of an's two systems
  const Analysis &og = order ? *order : an;
  std::vector<int> vl, vu;
  if (split) {
    vl.resize(n);
    vu.resize(n);
    for (int i = 0; i < n; i++) {
      vl[i] = virtual_rows(an.Lrp[i + 1] - an.Lrp[i] - 1, nr);
      vu[i] = virtual_rows(an.Ltrp[i + 1] - an.Ltrp[i] - 1, nr);
    }
  }
  std::vector<int> co[3];
  const int ncls = dag_coords(og, co);
  rows.resize(n);
  for (int i = 0; i < n; i++) rows[i] = i;
  pstart.assign(1, 0);
  Bisect bi(an, cap, rows, pstart);
  if (split) {
    bi.vl = &vl;
    bi.vu = &vu;
  }
  for (int c = 0; c < ncls; c++) bi.coord.push_back(&co[c]);
  bi.coord.push_back(&og.levL.level);
  bi.stamp_in.assign(n, 0);
  bi.stamp_l.assign(n, 0);
  bi.stamp_u.assign(n, 0);
  bi.side.assign(n, 0);
  bi.run(0, n);
  return bi.ok;
}

void block_schedule(const Analysis &an, bool lower, const std::vector<int> &rows, const std::vector<int> &pstart,
                    BlockSched &bs, bool split, int nr) {
  const int n = an.n;
  const std::vector<int> &rp = lower ? an.Lrp : an.Ltrp;
  const std::vector<int> &ci = lower ? an.Lci : an.Ltci;
  const std::vector<int> &glev = lower ? an.levL.level : an.levLt.level;
  const std::vector<int> &bylev = lower ? an.levL.rows : an.levLt.rows;
  const int nb = (int)pstart.size() - 1;
  auto deps = [&](int i, int &e0, int &e1) {
    e0 = lower ? rp[i] : rp[i] + 1;
    e1 = lower ? rp[i + 1] - 1 : rp[i + 1];
  };
  // Items: the rows (ids 0..n-1) and, for a split schedule, virtual rows (ids n..): a
  // row with m > nr dependencies keeps its nr-1 last-arriving ones plus the partial
  // sum of the rest, which a chain of virtual rows computes (the first sums nr
  // dependencies, each further one the previous partial and nr-1 more).  A virtual
  // row has right-hand side 0 and diagonal 1, so its value is -sum L_ij x_j, and its
  // consumer reads it with weight -1 (valmap -2).  Edges list (source item, factor
  // position or -2); each row's dependencies are in the order their values appear
  // (ascending level, ties by position), so a long row consumes its entries as they
  // arrive and the last to arrive is read last.
  std::vector<int> rptr(n + 1, 0), rsrc, rval;
  std::vector<int> vptr(1, 0), vsrc, vval, vown, vsub;
  std::vector<int> order;
  rsrc.reserve(rp[n]);
  rval.reserve(rp[n]);
  for (int i = 0; i < n; i++) {
    int e0, e1;
    deps(i, e0, e1);
    order.resize(e1 - e0);
    for (int q = e0; q < e1; q++) order[q - e0] = q;
    std::sort(order.begin(), order.end(), [&](int a, int c) {
      return glev[ci[a]] != glev[ci[c]] ? glev[ci[a]] < glev[ci[c]] : a < c;
    });
    const int m = e1 - e0;
    const int nv = split ? virtual_rows(m, nr) : 0;
    int own0 = 0;  // first of the row's own entries in `order`
    if (nv > 0) {
      const int c = m - (nr - 1);  // entries summed by the chain
      int at = 0, prev = -1;
      for (int v = 0; v < nv; v++) {
        const int id = n + (int)vown.size();
        const int take = std::min(c - at, v == 0 ? nr : nr - 1);
        if (prev >= 0) {
          vsrc.push_back(prev);
          vval.push_back(-2);
        }
        for (int t = 0; t < take; t++) {
          vsrc.push_back(ci[order[at + t]]);
          vval.push_back(order[at + t]);
        }
        at += take;
        vptr.push_back((int)vsrc.size());
        vown.push_back(i);
        vsub.push_back(v);
        prev = id;
      }
      rsrc.push_back(prev);
      rval.push_back(-2);
      own0 = c;
    }
    for (int t = own0; t < m; t++) {
      rsrc.push_back(ci[order[t]]);
      rval.push_back(order[t]);
    }
    rptr[i + 1] = (int)rsrc.size();
  }
  const int nvirt = (int)vown.size();
  const int nitem = n + nvirt;
  auto edges = [&](int it, const int *&src, const int *&val, int &cnt) {
    if (it < n) {
      src = rsrc.data() + rptr[it];
      val = rval.data() + rptr[it];
      cnt = rptr[it + 1] - rptr[it];
    } else {
      const int v = it - n;
      src = vsrc.data() + vptr[v];
      val = vval.data() + vptr[v];
      cnt = vptr[v + 1] - vptr[v];
    }
  };
  // levels of the item graph (the rows' levels when nothing is split), rows in level order
  std::vector<int> lx(nitem, 0), vfirst(n, -1);
  for (int v = nvirt - 1; v >= 0; v--) vfirst[vown[v]] = v;
  for (int i : bylev) {
    if (vfirst[i] >= 0)
      for (int v = vfirst[i]; v < nvirt && vown[v] == i; v++) {
        const int *src, *val;
        int cnt;
        edges(n + v, src, val, cnt);
        int l = 0;
        for (int e = 0; e < cnt; e++) l = std::max(l, lx[src[e]] + 1);
        lx[n + v] = l;
      }
    const int *src, *val;
    int cnt;
    edges(i, src, val, cnt);
    int l = 0;
    for (int e = 0; e < cnt; e++) l = std::max(l, lx[src[e]] + 1);
    lx[i] = l;
  }
  auto owner = [&](int it) { return it < n ? it : vown[it - n]; };
  bs.item_levels = 0;
  for (int it = 0; it < nitem; it++) bs.item_levels = std::max(bs.item_levels, lx[it] + 1);
  bs.n = n;
  bs.nr = nr;
  bs.nblocks = nb;
  bs.bptr.assign(nb + 1, 0);
  bs.brows.assign(nb, 0);
  bs.nreal.assign(nb, 0);
  auto src_of = [&](int b) { return lower ? b : nb - 1 - b; };
  std::vector<int> nvb(nb, 0);
  {
    std::vector<int> pb(n, 0);
    for (int b = 0; b < nb; b++)
      for (int t = pstart[b]; t < pstart[b + 1]; t++) pb[rows[t]] = b;
    for (int v = 0; v < nvirt; v++) nvb[pb[vown[v]]]++;
  }
  for (int b = 0; b < nb; b++) {
    const int s = src_of(b);
    bs.nreal[b] = pstart[s + 1] - pstart[s];
    bs.brows[b] = bs.nreal[b] + nvb[s];
    bs.bptr[b + 1] = bs.bptr[b] + (bs.brows[b] + 63) / 64 * 64;
  }
  const int npad = bs.bptr[nb];
  bs.npad = npad;
  bs.perm.assign(npad, -1);
  bs.diagmap.assign(npad, 0);
  std::vector<int> item(npad, -1);  // item of rank k
  std::vector<int> rank(nitem, 0), blk(nitem, 0);
  bs.max_local_levels = 0;
  {
    std::vector<std::vector<int>> vof(nb);
    std::vector<int> pb(n, 0);
    for (int b = 0; b < nb; b++)
      for (int t = pstart[b]; t < pstart[b + 1]; t++) pb[rows[t]] = b;
    for (int v = 0; v < nvirt; v++) vof[pb[vown[v]]].push_back(n + v);
    for (int b = 0; b < nb; b++) {
      const int s = src_of(b);
      std::vector<int> ord(rows.begin() + pstart[s], rows.begin() + pstart[s + 1]);
      ord.insert(ord.end(), vof[s].begin(), vof[s].end());
      // by level, ties in solve order of the owning rows, partials before their row
      std::sort(ord.begin(), ord.end(), [&](int a, int c) {
        if (lx[a] != lx[c]) return lx[a] < lx[c];
        const int oa = owner(a), oc = owner(c);
        if (oa != oc) return lower ? oa < oc : oa > oc;
        const int sa = a < n ? INT32_MAX : vsub[a - n], sc = c < n ? INT32_MAX : vsub[c - n];
        return sa < sc;
      });
      for (int t = 0; t < (int)ord.size(); t++) {
        const int it = ord[t], k = bs.bptr[b] + t;
        item[k] = it;
        rank[it] = k;
        blk[it] = b;
        if (it < n) {
          bs.perm[k] = it;
          bs.diagmap[k] = lower ? rp[it + 1] - 1 : rp[it];
        } else {
          bs.diagmap[k] = -1;  // diagonal 1
        }
      }
      if (!ord.empty()) bs.max_local_levels = std::max(bs.max_local_levels, lx[ord.back()] - lx[ord.front()] + 1);
    }
  }
  // ELL slices of 64 ranks for the dependencies beyond nr
  bs.nslices = npad / 64;
  bs.slice_ptr.assign(bs.nslices + 1, 0);
  bs.slice_nnz.assign(bs.nslices, 0);
  bs.cnt.assign(npad, 0);
  for (int k = 0; k < npad; k++) {
    if (item[k] < 0) continue;
    const int *src, *val;
    int cnt;
    edges(item[k], src, val, cnt);
    bs.cnt[k] = cnt;
    bs.slice_nnz[k / 64] = std::max(bs.slice_nnz[k / 64], cnt - nr);
  }
  for (int sl = 0; sl < bs.nslices; sl++) bs.slice_ptr[sl + 1] = bs.slice_ptr[sl] + 64 * bs.slice_nnz[sl];
  // bit 30 of cnt flags the ranks of slices that hold rows longer than nr
  for (int k = 0; k < npad; k++)
    if (bs.slice_nnz[k / 64] > 0) bs.cnt[k] |= kLongSlice;
  bs.ell = bs.slice_ptr[bs.nslices];
  bs.ref.assign(bs.ell, INT32_MIN);
  bs.valmap.assign(bs.ell, -1);
  bs.ref4.assign((size_t)nr * npad, INT32_MIN);
  bs.valmap4.assign((size_t)nr * npad, -1);
  // imports in order of first use, LDS slots
  bs.iptr.assign(nb + 1, 0);
  bs.irow.clear();
  bs.max_lds = 0;
  std::vector<int> imp_blk(n, -1), imp_slot(n, 0);
  for (int b = 0; b < nb; b++) {
    int nimp = 0;
    for (int k = bs.bptr[b]; k < bs.bptr[b] + bs.brows[b]; k++) {
      const int *src, *val;
      int cnt;
      edges(item[k], src, val, cnt);
      const int sl = k / 64, lane = k % 64;
      for (int e = 0; e < cnt; e++) {
        const int j = src[e];
        int slot;
        if (blk[j] == b) {
          slot = rank[j] - bs.bptr[b];
        } else {  // only rows are imported: a virtual row lives in its owner's block
          if (imp_blk[j] != b) {
            imp_blk[j] = b;
            imp_slot[j] = nimp++;
            bs.irow.push_back(j);
          }
          slot = bs.brows[b] + imp_slot[j];
        }
        if (e < nr) {
          bs.ref4[(size_t)e * npad + k] = -slot - 1;
          bs.valmap4[(size_t)e * npad + k] = val[e];
        } else {
          const int at = bs.slice_ptr[sl] + 64 * (e - nr) + lane;
          bs.ref[at] = -slot - 1;
          bs.valmap[at] = val[e];
        }
      }
    }
    bs.iptr[b + 1] = bs.iptr[b] + nimp;
    // unused register-cached entries read the block's zero slot (value 0, weight 0)
    const int zero = -(bs.brows[b] + nimp) - 1;
    for (int k = bs.bptr[b]; k < bs.bptr[b + 1]; k++)
      for (int q = 0; q < nr; q++)
        if (bs.ref4[(size_t)q * npad + k] == INT32_MIN) bs.ref4[(size_t)q * npad + k] = zero;
    bs.max_lds = std::max(bs.max_lds, bs.brows[b] + nimp + 1);
  }
  bs.nimp = bs.iptr[nb];
  // exports: imported rows, numbered block by block in rank order
  std::vector<int> exp_id(n, -1);
  for (int e = 0; e < bs.nimp; e++) exp_id[bs.irow[e]] = 0;
  bs.eptr.assign(nb + 1, 0);
  bs.erank.clear();
  for (int b = 0; b < nb; b++) {
    for (int k = bs.bptr[b]; k < bs.bptr[b] + bs.brows[b]; k++)
      if (bs.perm[k] >= 0 && exp_id[bs.perm[k]] == 0) {
        exp_id[bs.perm[k]] = (int)bs.erank.size() + 1;  // 1-based while numbering
        bs.erank.push_back(k - bs.bptr[b]);
      }
    bs.eptr[b + 1] = (int)bs.erank.size();
  }
  bs.nexp = (int)bs.erank.size();
  bs.isrc.resize(bs.nimp);
  for (int e = 0; e < bs.nimp; e++) bs.isrc[e] = exp_id[bs.irow[e]] - 1;
  // output order: each block's rows by increasing row index, then its virtual rows (row -1)
  bs.orow.assign(npad, 0);
  bs.oslot.assign(npad, 0);
  for (int b = 0; b < nb; b++) {
    std::vector<std::pair<int, int>> o, v;
    o.reserve(bs.nreal[b]);
    for (int t = 0; t < bs.brows[b]; t++) {
      const int r = bs.perm[bs.bptr[b] + t];
      if (r >= 0) o.push_back({r, t});
      else v.push_back({-1, t});
    }
    std::sort(o.begin(), o.end());
    o.insert(o.end(), v.begin(), v.end());
    for (int t = 0; t < bs.brows[b]; t++) {
      bs.orow[bs.bptr[b] + t] = o[t].first;
      bs.oslot[bs.bptr[b] + t] = o[t].second;
    }
  }
}

}  // namespace bnx
