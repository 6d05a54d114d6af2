// Internal declarations of the bnx library (not part of the C-ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>
#include <string>
#include <vector>

namespace bnx {

constexpr int kMaxP = 32;      // eigenpairs per solve
constexpr int kMaxK = 16;      // BFGS window
constexpr int kMaxQ = kMaxP + 1;
constexpr int kMaxVec = 80;    // vectors in one kernel argument list
constexpr int kJdMax = 16;     // largest Jacobi-Davidson search space
constexpr int kDacgStall = 200;  // float DACG: iterations without a 10 % gain that end it near tau
#ifndef BNX_NBMAX
#define BNX_NBMAX 1024
#endif
// Blocks of a streaming kernel, hence partials per dot for the single-workgroup control kernels to reduce.
// Measured end to end on the 100^3 diffusion eigensolve (fp64 leg): 512 -> 2.96, 1024 -> 3.12, 2048 -> 3.05
// eigenpairs/s (fewer blocks slow the SpMV, more make every control kernel read more partials).
constexpr int kNBMax = BNX_NBMAX;
constexpr int kPartSlots = 80; // dots per partial area
constexpr int kAreas = 11;     // partial areas; the last is for reductions run by their producer's last block
constexpr int kBlock = 256;
constexpr int kProbeHopsMax = 65536;  // longest chain of the latency probes

// Pointer list passed by value to kernels.
template <typename T>
struct VList {
  const T *p[kMaxVec];
};

// Scalars of the solve kept on the device (all in double).
struct DevCtl {
  // correction-equation PCG (Sec. 4.3)
  double theta, rho, gamma, beta, g0, gn, pJp, q, xx, xAx, eigres, gc0;
  double a[kMaxK], b[kMaxK], e[kMaxK], sig[kMaxK], rhoR[kMaxK];
  double zy[kMaxQ], zQ[kMaxQ], Qg[kMaxQ], Qc0[kMaxQ], Qp[kMaxQ], Qr[kMaxQ];
  double alpha[kMaxK];            // s_t^T r_t, chronological
  double M[kMaxK * kMaxK];        // M[s*kMaxK+t] = s_s^T r_t
  double QS[kMaxQ * kMaxK];       // QS[c*kMaxK+s] = q_c^T s_s
  double tol_pcg, tau, xi;
  int k, m, itmax, exit_rule, its, done, reason, first, eigtest;
  // DACG (Sec. 4.1)
  double dq, dxx, dxAx, dgamma, dgamma_prev, dalpha, dinv, dgn, dtol;
  int dits, ddone, ditmax;
  double dbest;                     // smallest ||g||/||x|| so far
  int dbest_it, dstall, dstalled;   // its iteration; stall window (0: off); set when the window ended it
  // outer step (always double)
  double oz[kMaxQ], onrm2, otheta, orn, oalpha, osn2, ornold;
  double oya, oyn2;  // s^T (r_k - r_{k+1}) and ||r_k - r_{k+1}||^2 for the full BFGS pair
  // Jacobi-Davidson search space (Sec. 6): H = V^T A V (row-major), Ritz values ascending, Ritz
  // vectors of H (vector c at jY[c*kJdMax ...], the coefficients of the c-th Ritz vector in V)
  double jH[kJdMax * kJdMax], jY[kJdMax * kJdMax], jev[kJdMax];
  // backward
  double bz[kMaxQ];
  int err;  // bounded wait exceeded somewhere
};

struct Buf {
  void *p = nullptr;
  size_t bytes = 0;
};

// Level schedule of a triangular factor.
struct Levels {
  int nlev = 0;
  std::vector<int> level;  // n: level of each row
  std::vector<int> ptr;   // nlev+1
  std::vector<int> rows;  // n, rows sorted by level
  int max_rows = 0;
};

// Block schedule of one triangular solve (LDS-staged sync-free solve).
// The rows are partitioned into blocks (partition_rows); the block order is a
// topological order of the solve's dependency graph, and inside a block the
// rows are sorted by their level in the whole graph.  A row's rank k is its
// index in that order: block b occupies ranks bptr[b] .. bptr[b]+brows[b]-1,
// padded up to a multiple of 64 (padding ranks: cnt 0, perm -1).
// A block keeps every value it reads in LDS: its own rows at their local rank,
// and the rows it needs from earlier blocks ("imports": iptr[b] .. iptr[b+1]-1,
// in order of first use) at brows[b] + import index, followed by one slot that
// holds 0.  Rows read by later blocks ("exports") travel through a compact
// buffer: block b publishes its exports, in rank order, at export ids
// eptr[b] .. eptr[b+1]-1 (erank: their local ranks), and an import names the
// export id it reads (isrc).  The solution itself is written once per block,
// in row order: orow / oslot list the block's rows by increasing row index with
// their local ranks.  The first kNR dependencies of
// rank k are at [q * npad + k] of ref4 / valmap4 (q < kNR), encoded as
// -(LDS slot)-1; unused ones point at the zero slot with valmap -1 (weight 0),
// so a row always reads kNR values.  Further dependencies of long rows are
// stored as 64-rank ELL slices: entry e >= kNR of lane l of slice s is at
// slice_ptr[s] + 64 (e - kNR) + l (ELL padding: ref INT_MIN, valmap -1).
constexpr int kNR = 4;   // dependency slots per row in registers (block solve)
constexpr int kNRC = 6;  // the same for level-compressed systems
constexpr int kNRW = 8;  // wide rows (split schedules of factors with many dependencies per row)
constexpr int kLongSlice = 1 << 30;  // flag in cnt: the rank's slice has rows longer than kNR
// LDS values per block (rows + imports + the zero slot, then the right-hand side of the block's ranks):
// 159 KiB of the 160 KiB of a CU.  The partition keeps rows + imports + zero slot within half of it.
constexpr int kLdsCap64 = 20352;
constexpr int kLdsCap32 = 40704;
// default LDS values per block of the partition (measured on the 7-point 100^3 grid)
constexpr int kBlkTarget64 = 7168;
constexpr int kBlkTarget32 = 12288;
constexpr int kBlkTarget32C = 8192;  // FP32, level-compressed systems: 256 blocks on the 100^3 grid
// level-pair substitution is tried for factors whose levels hold fewer rows than this on average
constexpr double kLpsRowsPerLevel = 512.0;

struct BlockSched {
  int n = 0, npad = 0, nblocks = 0, nslices = 0, ell = 0, nimp = 0;
  int nr = kNR;                // dependency slots per rank (kNR or kNRC)
  int max_local_levels = 0, max_lds = 0;
  int item_levels = 0;          // levels of the item graph (rows and virtual rows)
  std::vector<int> bptr;       // nblocks+1: first (padded) rank of each block
  std::vector<int> brows;      // nblocks: LDS rows of each block (its rows, then their virtual rows)
  std::vector<int> nreal;      // nblocks: rows of each block that are rows of the matrix
  std::vector<int> iptr;       // nblocks+1: imports of each block
  std::vector<int> irow;       // imported rows (original ids), in order of first use
  std::vector<int> isrc;       // export id of each import
  std::vector<int> eptr;       // nblocks+1: exports of each block
  std::vector<int> erank;      // local rank of each export
  std::vector<int> orow, oslot;  // npad: rows of each block by increasing row index (then -1 for virtual
                                 // rows), and their local ranks
  int nexp = 0;
  std::vector<int> perm;       // npad: original row of rank k (-1: padding or a virtual row)
  std::vector<int> diagmap;    // npad: factor value index of the diagonal of row perm[k] (-1: diagonal 1)
  std::vector<int> cnt;        // npad: number of dependencies of rank k (| kLongSlice)
  std::vector<int> ref4;       // kNR * npad
  std::vector<int> valmap4;    // kNR * npad, -1 where unused, -2 for weight -1 (a partial sum)
  std::vector<int> slice_ptr;  // nslices+1
  std::vector<int> slice_nnz;  // nslices: entries beyond kNR
  std::vector<int> ref;        // ell entries
  std::vector<int> valmap;     // ell entries: factor value index, -1 for padding
};

// Host-side analysis of the CSR pattern (done once per context).
struct Analysis {
  int n = 0, nnz = 0, nnzL = 0;
  std::vector<int> rp, ci;          // A
  std::vector<int> Lrp, Lci, mapL;  // L rows (diag last), A position of each L entry
  std::vector<int> Ltrp, Ltci, mapLt;  // L^T rows (diag first), L position of each L^T entry
  Levels levL, levLt;
};

// One direction's triangular system as the solves see it: rows of L for the forward
// solve (dependencies, then the diagonal), rows of L^T for the backward one (the
// diagonal, then the dependencies).  Its values come from that direction's factor
// values v (L, or L^T, in CSR):
//   entry e = (direct[e] >= 0 ? v[direct[e]] : 0) - sum_t v[ta[t]] v[tb[t]] / v[tc[t]],  t in [tp[e], tp[e+1]),
// and the right-hand side is transformed first: b'_i = b_i - sum_t (v[ma[t]] / v[mc[t]]) b_{mj[t]},
// t in [mp[i], mp[i+1]).  Level-pair substitution fills these (compress_system).
struct SolveSys {
  int n = 0, nnz = 0, nlev = 0;
  std::vector<int> rp, ci, direct, tp, ta, tb, tc;
  std::vector<int> mp, mj, ma, mc;
  std::vector<int> level;
};
// Level-pair substitution: every row on an even level has each dependency on an odd
// level replaced by that row's own equation, so it depends on rows further down and
// the chain of dependent levels roughly halves (the solution is unchanged up to
// rounding).  Returns false, leaving S unusable, when the levels do not drop below
// 3/4, a row would have more than maxdeps dependencies, or the system more than
// max_entries entries (diagonal included).
bool compress_system(const Analysis &an, bool lower, int maxdeps, SolveSys &S, long long max_entries = LLONG_MAX);
// The two compressed systems the fp32 solves use, when level-pair substitution pays: every row
// within kNRC dependencies, or (split schedules) longer rows with at most 1.5x the factor's entries.
bool compress_both(const Analysis &an, bool split, SolveSys &Sf, SolveSys &Sb);
// Level sets from per-row levels.
void levels_from(int n, const std::vector<int> &lev, Levels &L);
// Register slots of the block solve for the two systems of an analysis: 3 when no row of
// either has more than three dependencies (each slot costs a load per polling round),
// else kNR, or kNRC for level-compressed systems.
int slots_for(const Analysis &sys, bool compressed);

// Validate CSR; returns empty string if fine, else the problem.
std::string validate_csr(int n, int nnz, const int *rp, const int *ci);
// Build L / L^T patterns and level schedules.
void analyse(Analysis &an);
// Partition of the rows into blocks of at most cap LDS values each (the block's
// rows plus the distinct rows it reads from other blocks, in either solve
// direction).  Blocks are rows[pstart[b] .. pstart[b+1]-1], listed in a
// topological order of the forward graph.  Returns false when a single row
// does not fit.
// split: rows with more than kNR dependencies in either direction are solved
// through chains of virtual partial-sum rows (block_schedule), which take LDS
// slots of their own.
// order: when the two solve systems of an are not transposes of each other (level-pair
// substitution), the analysis of the factor they were derived from, whose coordinates are
// monotone along the dependencies of both.
bool partition_rows(const Analysis &an, int cap, std::vector<int> &rows, std::vector<int> &pstart, bool split,
                    int nr, const Analysis *order = nullptr);
// Virtual partial-sum rows a row with `deps` dependencies takes in a split schedule with nr slots.
int virtual_rows(int deps, int nr);
// Block schedule of the forward (lower = true: rows of L, diag last) or backward
// (rows of L^T, diag first) solve over a partition from partition_rows (the
// backward solve takes its blocks in reverse order).
void block_schedule(const Analysis &an, bool lower, const std::vector<int> &rows, const std::vector<int> &pstart,
                    BlockSched &bs, bool split, int nr);

// IC(lfil, tau_IC) factor of A + shift diag(A) (Sec. 2 initial preconditioner) in
// CSR, rows with ascending columns and the diagonal last.  The dropping rule is
// spelled out in ict.hip.  Returns false on a non-positive pivot.
struct IctFactor {
  std::vector<int> rp, ci;
  std::vector<double> v;
};
bool ict_factor(int n, const int *rp, const int *ci, const double *val, int lfil, double tau, double shift,
                IctFactor &L);
// Analysis input (the symmetric pattern L + L^T) whose tril is the pattern of L.
void pattern_of_factor(int n, const IctFactor &L, Analysis &an);

// ----------------------------------------------------------------- launchers
int spmv_group(double mean_nnz);

template <typename T>
struct Mat {
  int n = 0;
  const int *rp = nullptr, *ci = nullptr;
  const T *v = nullptr;
  int group = 8;
  // SELL-64 copy (used when present): slice s holds rows 64s..64s+63, entry e of
  // lane l at ell_ptr[s] + 64 e + l; padding has column = row and value 0.
  const int *ell_ptr = nullptr, *ell_len = nullptr, *ell_col = nullptr;
  const T *ell_val = nullptr;
};

// Device copy of a BlockSched with values of precision T.
template <typename T>
struct DevBlk {
  int n = 0, npad = 0, nblocks = 0;
  int nr = kNR;           // dependency slots per rank (kNR, or kNRC for a level-compressed system)
  int nexp = 0, ell = 0;  // ell: entries in the ELL slices (0: no row has more than kNR dependencies)
  const int *bptr = nullptr, *brows = nullptr, *iptr = nullptr, *isrc = nullptr;
  const int *eptr = nullptr, *erank = nullptr, *orow = nullptr, *oslot = nullptr;
  const int *perm = nullptr, *slice_ptr = nullptr, *slice_nnz = nullptr, *ref = nullptr;
  const int *cnt = nullptr, *ref4 = nullptr;
  const T *diag = nullptr, *val = nullptr, *val4 = nullptr;  // diag holds reciprocals
  // right-hand-side transform of a level-compressed system in rank order (mw slots per rank): slot e of
  // rank k names the substituted row mjr[e*npad + k] (-1: none) and its weight's index mtr[e*npad + k]
  // into the system's transform values
  const int *mjr = nullptr, *mtr = nullptr;
  int mw = 0;
};

// b'_i = b_i - sum_t mv[t] b_{mj[t]}, t in [mp[i], mp[i+1])
template <typename T>
struct RhsT {
  const int *mp = nullptr, *mj = nullptr;
  const T *mv = nullptr;
};

template <typename T>
struct Tri {
  DevBlk<T> blk;
  // Export buffer of the block solves of this precision, two halves of blk_nexp values, and their two
  // ticket counters.  A launch uses half (seq & 1) and resets the other half to the sentinel (and its
  // counter to 0) for the next launch of this precision, which always uses that other half.
  T *blk_exp = nullptr;
  int blk_nexp = 0;
  int *blk_cnt = nullptr;
  long long *blk_seq = nullptr;  // host: block-solve launches of this precision so far
  int n = 0;
  const int *rp = nullptr, *ci = nullptr;
  const T *v = nullptr;
  const int *lev_rows = nullptr;
  const std::vector<int> *lev_ptr = nullptr;  // level boundaries for level launches (host, owned by the context)
  int nlev = 0;
  int max_rows = 0;          // largest level
  bool lower = true;         // true: diag last (L); false: diag first (L^T)
  RhsT<T> M;                 // right-hand-side transform of a level-compressed system (none: mp null)
};

// Optional HIP-event timing of the SpMV and triangular-solve launches.
// Kernel ids: 0/1 SpMV fp64/fp32, 2/3 forward solve fp64/fp32, 4/5 backward solve fp64/fp32.
struct Profiler {
  static constexpr int kIds = 6;
  bool on = false;
  double ms[kIds] = {0};
  long long count[kIds] = {0};
  std::vector<hipEvent_t> pool;
  struct Pending {
    int id;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    (void)hipEventCreate(&e);
    return e;
  }
  void begin(hipStream_t st, hipEvent_t *a) {
    *a = get();
    (void)hipEventRecord(*a, st);
  }
  void end(hipStream_t st, int id, hipEvent_t a) {
    hipEvent_t b = get();
    (void)hipEventRecord(b, st);
    pending.push_back({id, a, b});
  }
  // call after the stream has been synchronised
  void drain() {
    for (auto &p : pending) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) {
        ms[p.id] += t;
        count[p.id]++;
      }
      pool.push_back(p.a);
      pool.push_back(p.b);
    }
    pending.clear();
  }
  void reset() {
    drain();
    for (int i = 0; i < kIds; i++) {
      ms[i] = 0;
      count[i] = 0;
    }
  }
  ~Profiler() {
    for (auto &p : pending) {
      pool.push_back(p.a);
      pool.push_back(p.b);
    }
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

struct Launch {
  Profiler *prof = nullptr;
  hipStream_t st;
  int nb;          // streaming blocks
  DevCtl *ctl;
  double *part;    // partial areas: area a at part + a*kPartSlots*kNBMax
  int *counter;    // work counters for sync-free solves
  int trsv_mode;
  int sf_waves;    // persistent waves for sync-free solves
};

inline double *area(const Launch &L, int a) { return L.part + (size_t)a * kPartSlots * kNBMax; }

template <typename T>
int launch_spmv(const Launch &L, const Mat<T> &A, const T *x, T *y, int ndy, const VList<T> &ly, int ndx,
                 const VList<T> &lx, double *part, const int *gate);
template <typename T, typename Acc>
int launch_multidot(const Launch &L, int n, int D, const VList<T> &X, const VList<T> &Y, double *part,
                    const int *gate);
// Dots of A_0 (and A_1 when na = 2) with each of V_0..V_{nv-1}, then A_0^T A_1 when ab = 1; partial order
// A_0^T V (nv), A_1^T V (nv), A_0^T A_1.  Returns the number of blocks (partials per dot).
template <typename T, typename Acc>
int launch_mdot_list(const Launch &L, int n, int na, const T *A0, const T *A1, int nv, const VList<T> &V, int ab,
                     double *part, const int *gate);
int grid_for(size_t work, int nbmax);
template <typename T>
void launch_trsv(const Launch &L, const Tri<T> &F, const T *b, T *x, int kfuse, const VList<T> &R,
                 const double *coef, const int *gate);
template <typename Tin, typename Tout>
void launch_cast(hipStream_t st, size_t n, const Tin *in, Tout *out);
template <typename T>
void launch_fill(hipStream_t st, size_t n, T *x, T v);
// Both halves of a block-solve export buffer (2 * nexp_half values) to the sentinel, both ticket counters to 0.
template <typename T>
void launch_blk_reset(hipStream_t st, T *xe_pair, int nexp_half, int *cnt_pair);
// Latency probes (kind 0: LDS hand-over between waves, 1: global flag between workgroups).
void launch_probe(hipStream_t st, int kind, int hops, int *flags, int *counter, int *err);

}  // namespace bnx
