// Generic device kernels of the bnx library for gfx950 (wave64):
//   CSR SpMV with fused dot-product epilogue (the MVP of the paper's tables),
//   fused tall-skinny multi-dot, level-scheduled and sync-free triangular
//   solves for the IC(0) preconditioner P0^ = (L L^T)^{-1} (Sec. 2), casts, fills.
// Dot products are reduced deterministically: every block writes one partial
// per dot, and a single-block control kernel sums the partials in fixed order.
#include <cstdio>
#include <cstdlib>

#include "internal.h"

namespace bnx {

// ------------------------------------------------------------------ helpers
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Reduce ND per-thread accumulators over the block and write part[d*gridDim.x + blockIdx.x].
template <typename T, int MAXD>
__device__ __forceinline__ void block_partials(T (&acc)[MAXD], int nd, double *part) {
  __shared__ double red[kBlock / 64][MAXD];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int d = 0; d < MAXD; d++) {
    if (d < nd) {
      T s = wave_sum(acc[d]);
      if (lane == 0) red[w][d] = (double)s;
    }
  }
  __syncthreads();
  if (threadIdx.x < nd) {
    double s = 0.0;
#pragma unroll
    for (int ww = 0; ww < kBlock / 64; ww++) s += red[ww][threadIdx.x];
    part[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = s;
  }
}

int spmv_group(double mean) {
  int g = 1;
  while (g < 64 && g < mean) g <<= 1;
  return g;
}

int grid_for(size_t work, int nbmax) {
  size_t b = (work + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  if (b > (size_t)nbmax) b = nbmax;
  return (int)b;
}

// ------------------------------------------------------------------ SpMV
// y = A x with G lanes per row.  Epilogue dots (per block partials):
//   d <  ndy : sum_i y_i * ly[d][i]
//   d >= ndy : sum_i x_i * lx[d-ndy][i]
template <typename T, int G, int MAXD>
__global__ __launch_bounds__(kBlock) void k_spmv(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                                 const T *__restrict__ v, const T *__restrict__ x, T *__restrict__ y,
                                                 int ndy, VList<T> ly, int ndx, VList<T> lx, double *part,
                                                 const int *gate) {
  if (gate && *gate) return;
  const int lane = threadIdx.x % G;
  const int grp = (blockIdx.x * kBlock + threadIdx.x) / G;
  const int ngrp = gridDim.x * (kBlock / G);
  constexpr int NA = MAXD > 0 ? MAXD : 1;
  T acc[NA];
#pragma unroll
  for (int d = 0; d < NA; d++) acc[d] = T(0);
  for (int row = grp; row < n; row += ngrp) {
    T s = T(0);
    const int e1 = rp[row + 1];
    for (int e = rp[row] + lane; e < e1; e += G) s += v[e] * x[ci[e]];
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, G);
    if (lane == 0) {
      y[row] = s;
      if (MAXD > 0) {
        const T xr = x[row];
#pragma unroll
        for (int d = 0; d < MAXD; d++) {
          if (d < ndy) acc[d] += s * ly.p[d][row];
          else if (d < ndy + ndx) acc[d] += xr * lx.p[d - ndy][row];
        }
      }
    }
  }
  if (MAXD > 0) block_partials<T, NA>(acc, ndy + ndx, part);
}

template <typename T, int G>
static int spmv_dispatch_d(const Launch &L, const Mat<T> &A, const T *x, T *y, int ndy, const VList<T> &ly, int ndx,
                            const VList<T> &lx, double *part, const int *gate) {
  const int nd = ndy + ndx;
  const int nb = grid_for((size_t)A.n * G, kNBMax);
  if (nd == 0)
    hipLaunchKernelGGL((k_spmv<T, G, 0>), dim3(nb), dim3(kBlock), 0, L.st, A.n, A.rp, A.ci, A.v, x, y, 0, ly, 0, lx,
                       part, gate);
  else if (nd <= 6)
    hipLaunchKernelGGL((k_spmv<T, G, 6>), dim3(nb), dim3(kBlock), 0, L.st, A.n, A.rp, A.ci, A.v, x, y, ndy, ly, ndx,
                       lx, part, gate);
  else if (nd <= 24)
    hipLaunchKernelGGL((k_spmv<T, G, 24>), dim3(nb), dim3(kBlock), 0, L.st, A.n, A.rp, A.ci, A.v, x, y, ndy, ly, ndx,
                       lx, part, gate);
  else
    hipLaunchKernelGGL((k_spmv<T, G, 72>), dim3(nb), dim3(kBlock), 0, L.st, A.n, A.rp, A.ci, A.v, x, y, ndy, ly,
                       ndx, lx, part, gate);
  return nb;
}

// Number of blocks a SpMV launch uses (the control kernels need it).
// SELL-64 SpMV: one row per lane, column-major entries inside each 64-row
// slice, so value, column and (for banded matrices) x loads and the y store
// are coalesced.  Same epilogue dots as k_spmv, computed by every lane.
template <typename T, int MAXD>
__global__ __launch_bounds__(kBlock) void k_spmv_ell(int n, const int *__restrict__ eptr, const int *__restrict__ elen,
                                                     const int *__restrict__ ecol, const T *__restrict__ eval,
                                                     const T *__restrict__ x, T *__restrict__ y, int ndy, VList<T> ly,
                                                     int ndx, VList<T> lx, double *part, const int *gate) {
  if (gate && *gate) return;
  constexpr int NA = MAXD > 0 ? MAXD : 1;
  T acc[NA];
#pragma unroll
  for (int d = 0; d < NA; d++) acc[d] = T(0);
  for (int row = blockIdx.x * kBlock + threadIdx.x; row < n; row += gridDim.x * kBlock) {
    const int sl = row >> 6, lane = row & 63;
    const int base = eptr[sl] + lane, len = elen[sl];
    T s = T(0);
    // batches of 8 entries: all column and value loads issued before the x gathers
    for (int e0 = 0; e0 < len; e0 += 8) {
      int cc[8];
      T vv[8];
#pragma unroll
      for (int q = 0; q < 8; q++) {
        const bool ok = e0 + q < len;
        cc[q] = ok ? ecol[base + 64 * (e0 + q)] : row;
        vv[q] = ok ? eval[base + 64 * (e0 + q)] : T(0);
      }
      T xx[8];
#pragma unroll
      for (int q = 0; q < 8; q++) xx[q] = x[cc[q]];
#pragma unroll
      for (int q = 0; q < 8; q++) s += vv[q] * xx[q];
    }
    y[row] = s;
    if (MAXD > 0) {
      const T xr = x[row];
#pragma unroll
      for (int d = 0; d < NA; d++) {
        if (d < ndy) acc[d] += s * ly.p[d][row];
        else if (d < ndy + ndx) acc[d] += xr * lx.p[d - ndy][row];
      }
    }
  }
  if (MAXD > 0) block_partials<T, NA>(acc, ndy + ndx, part);
}

template <typename T>
static int spmv_switch(const Launch &L, const Mat<T> &A, const T *x, T *y, int ndy, const VList<T> &ly, int ndx,
                       const VList<T> &lx, double *part, const int *gate) {
  if (A.ell_ptr) {
    const int nd = ndy + ndx;
    const int nb = grid_for((size_t)A.n, kNBMax);
    if (nd == 0)
      hipLaunchKernelGGL((k_spmv_ell<T, 0>), dim3(nb), dim3(kBlock), 0, L.st, A.n, A.ell_ptr, A.ell_len, A.ell_col,
                         A.ell_val, x, y, 0, ly, 0, lx, part, gate);
    else if (nd <= 6)
      hipLaunchKernelGGL((k_spmv_ell<T, 6>), dim3(nb), dim3(kBlock), 0, L.st, A.n, A.ell_ptr, A.ell_len, A.ell_col,
                         A.ell_val, x, y, ndy, ly, ndx, lx, part, gate);
    else
      hipLaunchKernelGGL((k_spmv_ell<T, 72>), dim3(nb), dim3(kBlock), 0, L.st, A.n, A.ell_ptr, A.ell_len, A.ell_col,
                         A.ell_val, x, y, ndy, ly, ndx, lx, part, gate);
    return nb;
  }
  switch (A.group) {
    case 1: return spmv_dispatch_d<T, 1>(L, A, x, y, ndy, ly, ndx, lx, part, gate);
    case 2: return spmv_dispatch_d<T, 2>(L, A, x, y, ndy, ly, ndx, lx, part, gate);
    case 4: return spmv_dispatch_d<T, 4>(L, A, x, y, ndy, ly, ndx, lx, part, gate);
    case 8: return spmv_dispatch_d<T, 8>(L, A, x, y, ndy, ly, ndx, lx, part, gate);
    case 16: return spmv_dispatch_d<T, 16>(L, A, x, y, ndy, ly, ndx, lx, part, gate);
    case 32: return spmv_dispatch_d<T, 32>(L, A, x, y, ndy, ly, ndx, lx, part, gate);
    default: return spmv_dispatch_d<T, 64>(L, A, x, y, ndy, ly, ndx, lx, part, gate);
  }
}

template <typename T>
int launch_spmv(const Launch &L, const Mat<T> &A, const T *x, T *y, int ndy, const VList<T> &ly, int ndx,
                const VList<T> &lx, double *part, const int *gate) {
  const bool prof = L.prof && L.prof->on;
  hipEvent_t a = nullptr;
  if (prof) L.prof->begin(L.st, &a);
  const int nb = spmv_switch<T>(L, A, x, y, ndy, ly, ndx, lx, part, gate);
  if (prof) L.prof->end(L.st, sizeof(T) == 8 ? 0 : 1, a);
  return nb;
}

// ------------------------------------------------------------------ multi-dot
// part[d] = sum_i X[d][i] * Y[d][i] for d < D, one pass over the rows.
template <typename T, typename Acc, int MAXD>
__global__ __launch_bounds__(kBlock) void k_multidot(int n, int D, VList<T> X, VList<T> Y, double *part,
                                                     const int *gate) {
  if (gate && *gate) return;
  Acc acc[MAXD];
#pragma unroll
  for (int d = 0; d < MAXD; d++) acc[d] = Acc(0);
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
#pragma unroll
    for (int d = 0; d < MAXD; d++)
      if (d < D) acc[d] += (Acc)X.p[d][i] * (Acc)Y.p[d][i];
  }
  block_partials<Acc, MAXD>(acc, D, part);
}

template <typename T, typename Acc>
int launch_multidot(const Launch &L, int n, int D, const VList<T> &X, const VList<T> &Y, double *part,
                    const int *gate) {
  if (D <= 0) return 0;
  const int nb = grid_for((size_t)n, L.nb);
  if (D <= 4)
    hipLaunchKernelGGL((k_multidot<T, Acc, 4>), dim3(nb), dim3(kBlock), 0, L.st, n, D, X, Y, part, gate);
  else if (D <= 16)
    hipLaunchKernelGGL((k_multidot<T, Acc, 16>), dim3(nb), dim3(kBlock), 0, L.st, n, D, X, Y, part, gate);
  else if (D <= 48)
    hipLaunchKernelGGL((k_multidot<T, Acc, 48>), dim3(nb), dim3(kBlock), 0, L.st, n, D, X, Y, part, gate);
  else
    hipLaunchKernelGGL((k_multidot<T, Acc, kMaxVec>), dim3(nb), dim3(kBlock), 0, L.st, n, D, X, Y, part, gate);
  return nb;
}

// ------------------------------------------------------------------ triangular solves
// Right-hand side of row i: b_i - sum_t coef[t] * R[t][i]  (the w = g - R a of Alg. 1 fused in).
template <typename T>
__device__ __forceinline__ T rhs_value(int i, const T *b, int kfuse, const VList<T> &R, const double *coef) {
  T s = b[i];
  for (int t = 0; t < kfuse; t++) s -= (T)coef[t] * R.p[t][i];
  return s;
}

// One dependency level, one thread per row.  lower: x_i = (b_i - sum_{e<diag} L_e x_c)/L_diag (diag last);
// upper (rows of L^T): x_i = (b_i - sum_{e>diag} Lt_e x_c)/Lt_diag (diag first).
template <typename T, bool LOWER>
__global__ __launch_bounds__(kBlock) void k_trsv_level(int r0, int r1, const int *__restrict__ rows,
                                                       const int *__restrict__ rp, const int *__restrict__ ci,
                                                       const T *__restrict__ v, const T *__restrict__ b, T *x,
                                                       int kfuse, VList<T> R, const double *coef, const int *gate) {
  if (gate && *gate) return;
  int pos = r0 + blockIdx.x * kBlock + threadIdx.x;
  if (pos >= r1) return;
  const int i = rows[pos];
  T s = rhs_value(i, b, kfuse, R, coef);
  const int e0 = rp[i], e1 = rp[i + 1];
  T d;
  if (LOWER) {
    for (int e = e0; e < e1 - 1; e++) s -= v[e] * x[ci[e]];
    d = v[e1 - 1];
  } else {
    for (int e = e0 + 1; e < e1; e++) s -= v[e] * x[ci[e]];
    d = v[e0];
  }
  x[i] = s / d;
}

// Sentinel bit patterns (signalling NaNs never produced by arithmetic).
template <typename T>
struct Sentinel;
template <>
struct Sentinel<double> {
  using U = unsigned long long;
  static constexpr U bits = 0x7FF4DEAD7FF4DEADull;
};
template <>
struct Sentinel<float> {
  using U = unsigned int;
  static constexpr U bits = 0x7F8ADEADu;
};

template <typename T>
__device__ __forceinline__ typename Sentinel<T>::U to_bits(T v) {
  if constexpr (sizeof(T) == 8) return (unsigned long long)__double_as_longlong(v);
  else return (unsigned int)__float_as_uint(v);
}
template <typename T>
__device__ __forceinline__ T from_bits(typename Sentinel<T>::U u) {
  if constexpr (sizeof(T) == 8) return __longlong_as_double((long long)u);
  else return __uint_as_float(u);
}

// Fill x with the sentinel and reset the work counter.
template <typename T>
__global__ void k_sentinel(size_t n, T *x, int *counter, const int *gate) {
  if (gate && *gate) return;
  using U = typename Sentinel<T>::U;
  U *xu = reinterpret_cast<U *>(x);
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    xu[i] = Sentinel<T>::bits;
  if (blockIdx.x == 0 && threadIdx.x == 0) *counter = 0;
}

constexpr int kSpinLimit = 1 << 20;
// Block solve polling: LDS polling rounds between examinations of the external
// polls, and the s_sleep issued after a polling round without progress.
#ifndef BNX_TRSV_ILIM
#define BNX_TRSV_ILIM 2
#endif
#ifndef BNX_TRSV_SLEEP
#define BNX_TRSV_SLEEP 0
#endif
#ifndef BNX_TRSV_WC
#define BNX_TRSV_WC 12
#endif
#ifndef BNX_TRSV_PUBSLEEP
#define BNX_TRSV_PUBSLEEP 1
#endif

// Sync-free solve: a persistent grid of waves takes chunks of 64 rows in level
// order from a counter; a lane owns one row, consumes its dependencies as they
// appear (each x value doubles as its own completion flag: it leaves the
// sentinel state exactly once, written with a device-scope atomic store), and
// publishes x_i as soon as its last dependency arrived.  A chunk only depends
// on earlier chunks (rows are sorted by level) or on lanes of the same wave
// that finish inside the same polling loop, so progress is guaranteed.  Every
// wait is bounded; on overflow the row is written as NaN and ctl->err is set.
template <typename T, bool LOWER>
__global__ __launch_bounds__(kBlock) void k_trsv_sf(int n, const int *__restrict__ rows, const int *__restrict__ rp,
                                                    const int *__restrict__ ci, const T *__restrict__ v,
                                                    const T *__restrict__ b, T *x, int kfuse, VList<T> R,
                                                    const double *coef, int *counter, int *err, const int *gate) {
  if (gate && *gate) return;
  using U = typename Sentinel<T>::U;
  U *xu = reinterpret_cast<U *>(x);
  const int lane = threadIdx.x & 63;
  const int nchunks = (n + 63) >> 6;
  for (;;) {
    int chunk = 0;
    if (lane == 0) chunk = atomicAdd(counter, 1);
    chunk = __shfl(chunk, 0, 64);
    if (chunk >= nchunks) break;
    const int pos = (chunk << 6) + lane;
    if (pos < n) {
      const int i = rows[pos];
      T s = rhs_value(i, b, kfuse, R, coef);
      const int e0 = rp[i], e1 = rp[i + 1];
      int e, eend;
      T d;
      if (LOWER) {
        e = e0;
        eend = e1 - 1;
        d = v[e1 - 1];
      } else {
        e = e0 + 1;
        eend = e1;
        d = v[e0];
      }
      int spins = 0;
      bool fin = false;
      while (!fin) {
        while (e < eend) {
          U u = __hip_atomic_load(&xu[ci[e]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (u == Sentinel<T>::bits) break;
          s -= v[e] * from_bits<T>(u);
          e++;
        }
        if (e == eend) {
          __hip_atomic_store(&xu[i], to_bits<T>(s / d), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          fin = true;
        } else if (++spins > kSpinLimit) {
          __hip_atomic_store(&xu[i], to_bits<T>(T(__builtin_nan(""))), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          atomicOr(err, 1);
          fin = true;
        } else {
          __builtin_amdgcn_s_sleep(1);
        }
      }
    }
  }
}

// LDS-staged sync-free solve: one 1024-thread workgroup per block of B rows
// (taken in block order from a ticket counter).  The block's solution lives in
// LDS; in-block dependencies are read from LDS, external ones (earlier blocks)
// from the global solution, both polled until they leave the sentinel state.
// Each wave walks its 64-row slices of the block in order (rows sorted by local
// level), so a lane only waits on rows of lower rank, which finish first.
// Right-hand side in solve order and sentinel fill of the rank-ordered solution:
//   bp[k] = b[perm[k]] - sum_t coef[t] R_t[perm[k]],  xr[k] = sentinel,  counter = 0.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_trsv_prep(int n, const int *__restrict__ perm, const T *__restrict__ b,
                                                      int kfuse, VList<T> R, const double *coef, T *bp, T *xr,
                                                      int *counter, const int *gate) {
  if (gate && *gate) return;
  using U = typename Sentinel<T>::U;
  U *xu = reinterpret_cast<U *>(xr);
  for (int k = blockIdx.x * kBlock + threadIdx.x; k < n; k += gridDim.x * kBlock) {
    bp[k] = rhs_value(perm[k], b, kfuse, R, coef);
    xu[k] = Sentinel<T>::bits;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *counter = 0;
}

template <typename T, int NR>
struct RowPre {
  int cnt;
  T d, s;
  int rr[NR];
  T vv[NR];
};

// Row data of rank base+lane (all loads rank-indexed and independent of each other).
template <typename T, int NR>
__device__ __forceinline__ void row_fetch(const DevBlk<T> &F, const T *bp, int base, int k1, int lane,
                                          RowPre<T, NR> &R) {
  const int k = base + lane;
  const bool ok = k < k1;
  const int n = F.n;
  R.cnt = ok ? F.cnt[k] : 0;
  R.d = ok ? F.diag[k] : T(1);  // reciprocal of the diagonal
  R.s = ok ? bp[k] : T(0);
#pragma unroll
  for (int q = 0; q < NR; q++) {
    R.rr[q] = ok ? F.ref4[(size_t)q * n + k] : INT32_MIN;
    R.vv[q] = ok ? F.val4[(size_t)q * n + k] : T(0);
  }
}

// LDS-staged sync-free solve.  One 1024-thread workgroup per block of B ranks
// (blocks taken in order from a ticket counter); the block's solution lives in
// LDS, indexed by local rank.
//  * 12 compute waves walk the block's 64-row slices in order (wave w takes
//    slices w, w+12, ...).  A lane resolves its row's dependencies from LDS
//    (in-block) or by polling the rank-ordered global solution xr (earlier
//    blocks), and writes its result to LDS only, so compute waves never wait
//    on their own stores.
//  * 4 publisher waves copy finished LDS values to xr (coalesced, for later
//    blocks) and to the output x (original order).
// Every dependency has a lower rank, so the lowest unfinished row can always
// proceed.  Waits are bounded: on overflow the value becomes NaN and *err is set.
template <typename T, int B>
__global__ __launch_bounds__(1024) void k_trsv_blk(DevBlk<T> F, const T *__restrict__ bp, T *x, T *xr, int *counter,
                                                    int *err, const int *gate) {
  if (gate && *gate) return;
  using U = typename Sentinel<T>::U;
  constexpr int NR = kNR;  // dependencies cached in registers per row
  constexpr int WC = BNX_TRSV_WC;  // compute waves
  constexpr int WP = 16 - WC;
  __shared__ U xs[B];
  __shared__ int blk_s;
  if (threadIdx.x == 0) blk_s = atomicAdd(counter, 1);
  for (int i = threadIdx.x; i < B; i += 1024) xs[i] = Sentinel<T>::bits;
  __syncthreads();
  const int blk = blk_s;
  if (blk >= F.nblocks) return;
  U *xru = reinterpret_cast<U *>(xr);
  U *xu = reinterpret_cast<U *>(x);
  const int n = F.n;
  const int k0 = blk * B, k1 = (k0 + B < n) ? k0 + B : n;
  const int nsl = (k1 - k0 + 63) >> 6;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;

  if (wave >= WC) {  // publisher
    for (int sl = wave - WC; sl < nsl; sl += WP) {
      const int t = (sl << 6) + lane;
      const int k = k0 + t;
      if (k < k1) {
        const int row = F.perm[k];
        U u;
        int spins = 0;
        while ((u = __hip_atomic_load(&xs[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) == Sentinel<T>::bits) {
          if (++spins > kSpinLimit) {
            u = to_bits<T>(T(__builtin_nan("")));
            atomicOr(err, 1);
            break;
          }
          if (BNX_TRSV_PUBSLEEP > 0) __builtin_amdgcn_s_sleep(BNX_TRSV_PUBSLEEP);
        }
        __hip_atomic_store(&xru[k], u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        xu[row] = u;
      }
    }
    return;
  }

  // two rounds of row data in flight ahead of the current one
  RowPre<T, NR> cur, nx1, nx2;
  if (wave < nsl) row_fetch<T, NR>(F, bp, k0 + (wave << 6), k1, lane, nx1);
  if (wave + WC < nsl) row_fetch<T, NR>(F, bp, k0 + ((wave + WC) << 6), k1, lane, nx2);
  for (int sl = wave; sl < nsl; sl += WC) {
    const int base = k0 + (sl << 6);
    cur = nx1;
    nx1 = nx2;
    if (sl + 2 * WC < nsl) row_fetch<T, NR>(F, bp, k0 + ((sl + 2 * WC) << 6), k1, lane, nx2);
    const int t = base - k0 + lane;
    bool fin = base + lane >= k1;
    const int nown = cur.cnt < NR ? cur.cnt : NR;
    const int nlong = cur.cnt;  // entries beyond NR come from the ELL slices
    const int gsl = base >> 6;
    const int esp = nlong > NR ? F.slice_ptr[gsl] + lane : 0;
    unsigned need_l = 0, need_g = 0;
#pragma unroll
    for (int q = 0; q < NR; q++) {
      if (q < nown) {
        if (cur.rr[q] < 0) need_l |= 1u << q;
        else need_g |= 1u << q;
      }
    }
    T xv[NR];
#pragma unroll
    for (int q = 0; q < NR; q++) xv[q] = T(0);
    unsigned seen = 0;
    bool cached_done = false;
    T s = cur.s;
    int e = NR, spins = 0;
    while (!fin) {
      // 1) polls of external dependencies, examined after the LDS phase (skipped by the
      //    whole wave when no lane has one pending, so no memory wait is needed then)
      const bool gpend = (need_g & ~seen) != 0u;
      const bool anyg = __builtin_amdgcn_ballot_w64(gpend) != 0ull;
      U gv[NR];
      if (anyg) {
#pragma unroll
        for (int q = 0; q < NR; q++)
          gv[q] = ((need_g & ~seen) >> q & 1u)
                      ? __hip_atomic_load(&xru[cur.rr[q]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                      : Sentinel<T>::bits;
      }
      // 2) LDS phase; a row whose dependencies have all arrived finishes here
      for (int it = 0; it < BNX_TRSV_ILIM && !fin && (need_l & ~seen); it++, spins++) {
        const unsigned pend = need_l & ~seen;
        U lv[NR];
#pragma unroll
        for (int q = 0; q < NR; q++)  // all LDS polls issued before any result is examined
          lv[q] = (pend >> q & 1u)
                      ? __hip_atomic_load(&xs[-cur.rr[q] - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)
                      : Sentinel<T>::bits;
#pragma unroll
        for (int q = 0; q < NR; q++)
          if ((pend >> q & 1u) && lv[q] != Sentinel<T>::bits) {
            xv[q] = from_bits<T>(lv[q]);
            seen |= 1u << q;
          }
        if (BNX_TRSV_SLEEP > 0 && (need_l & ~seen) == pend) __builtin_amdgcn_s_sleep(BNX_TRSV_SLEEP);
        if (seen == (need_l | need_g) && nlong <= NR) {
#pragma unroll
          for (int q = 0; q < NR; q++) s -= cur.vv[q] * xv[q];
          __hip_atomic_store(&xs[t], to_bits<T>(s * cur.d), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          fin = true;
        }
      }
      if (fin) break;
      // 3) results of the external polls
      if (anyg) {
#pragma unroll
        for (int q = 0; q < NR; q++)
          if (((need_g & ~seen) >> q & 1u) && gv[q] != Sentinel<T>::bits) {
            xv[q] = from_bits<T>(gv[q]);
            seen |= 1u << q;
          }
      }
      if (seen == (need_l | need_g)) {
        if (!cached_done) {
#pragma unroll
          for (int q = 0; q < NR; q++) s -= cur.vv[q] * xv[q];
          cached_done = true;
        }
        // rows longer than the register cache: the remaining entries in order
        bool blocked = false;
        while (e < nlong) {
          const int at = esp + 64 * (e - NR);
          const int r = F.ref[at];
          const U u = r < 0 ? __hip_atomic_load(&xs[-r - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)
                            : __hip_atomic_load(&xru[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (u == Sentinel<T>::bits) {
            blocked = true;
            break;
          }
          s -= F.val[at] * from_bits<T>(u);
          e++;
        }
        if (!blocked) {
          __hip_atomic_store(&xs[t], to_bits<T>(s * cur.d), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          fin = true;
          break;
        }
      }
      if (++spins > kSpinLimit) {
        __hip_atomic_store(&xs[t], to_bits<T>(T(__builtin_nan(""))), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        atomicOr(err, 1);
        fin = true;
      } else if (!(need_l & ~seen)) {
        __builtin_amdgcn_s_sleep(1);  // only external dependencies left
      }
    }
  }
}

template <typename T>
constexpr int blk_rows() {
  return (128 * 1024) / (int)sizeof(T);
}
// Rows per block: the largest block whose solution fits 128 KiB of LDS, unless
// overridden (BNX_BLK_ROWS, a power of two from 1024 up to that size).
int block_rows_for(int elem_bytes) {
  const int mx = elem_bytes == 8 ? blk_rows<double>() : blk_rows<float>();
  if (const char *e = getenv("BNX_BLK_ROWS")) {
    const int v = atoi(e);
    if (v >= 1024 && v <= mx && (v & (v - 1)) == 0) return v;
  }
  return mx;
}

template <typename T, int B>
static void launch_blk(const Launch &L, const Tri<T> &F, const T *bp, T *x, T *xr, const int *gate) {
  hipLaunchKernelGGL((k_trsv_blk<T, B>), dim3(F.blk.nblocks), dim3(1024), 0, L.st, F.blk, bp, x, xr, L.counter,
                     &L.ctl->err, gate);
}

template <typename T>
void launch_trsv(const Launch &L, const Tri<T> &F, const T *b, T *x, int kfuse, const VList<T> &R,
                 const double *coef, const int *gate) {
  if (L.trsv_mode == 0 && F.blk.nblocks > 0) {
    const bool prof0 = L.prof && L.prof->on;
    hipEvent_t ev0 = nullptr;
    T *bp = reinterpret_cast<T *>(F.blk_scratch);
    T *xr = reinterpret_cast<T *>(F.blk_xr);
    hipLaunchKernelGGL((k_trsv_prep<T>), dim3(grid_for(F.n, kNBMax)), dim3(kBlock), 0, L.st, F.n, F.blk.perm, b, kfuse,
                       R, coef, bp, xr, L.counter, gate);
    if (prof0) L.prof->begin(L.st, &ev0);
    switch (F.blk.B) {
      case 1024: launch_blk<T, 1024>(L, F, bp, x, xr, gate); break;
      case 2048: launch_blk<T, 2048>(L, F, bp, x, xr, gate); break;
      case 4096: launch_blk<T, 4096>(L, F, bp, x, xr, gate); break;
      case 8192: launch_blk<T, 8192>(L, F, bp, x, xr, gate); break;
      case 16384: launch_blk<T, 16384>(L, F, bp, x, xr, gate); break;
      default: launch_blk<T, blk_rows<T>()>(L, F, bp, x, xr, gate); break;
    }
    if (prof0) L.prof->end(L.st, (F.lower ? 2 : 4) + (sizeof(T) == 8 ? 0 : 1), ev0);
    return;
  }
  const bool prof = L.prof && L.prof->on;
  const int pid = (F.lower ? 2 : 4) + (sizeof(T) == 8 ? 0 : 1);
  hipEvent_t ev = nullptr;
  if (L.trsv_mode == 1) {  // one launch per dependency level
    if (prof) L.prof->begin(L.st, &ev);
    for (int l = 0; l < F.nlev; l++) {
      int r0 = F.lev_ptr[l], r1 = F.lev_ptr[l + 1];
      int nb = (r1 - r0 + kBlock - 1) / kBlock;
      if (F.lower)
        hipLaunchKernelGGL((k_trsv_level<T, true>), dim3(nb), dim3(kBlock), 0, L.st, r0, r1, F.lev_rows, F.rp, F.ci,
                           F.v, b, x, kfuse, R, coef, gate);
      else
        hipLaunchKernelGGL((k_trsv_level<T, false>), dim3(nb), dim3(kBlock), 0, L.st, r0, r1, F.lev_rows, F.rp,
                           F.ci, F.v, b, x, kfuse, R, coef, gate);
    }
    if (prof) L.prof->end(L.st, pid, ev);
    return;
  }
  // In-flight window: about three levels' worth of 64-row chunks.  Waves beyond
  // that would only poll, and their polling traffic slows the dependency chain.
  const int nchunks = (F.n + 63) / 64;
  int waves = L.sf_waves > 0 ? L.sf_waves : 3 * ((F.max_rows + 63) / 64);
  if (waves < 16) waves = 16;
  if (waves > 2048) waves = 2048;
  if (waves > nchunks) waves = nchunks;
  int nb = (waves + 3) / 4;
  hipLaunchKernelGGL((k_sentinel<T>), dim3(grid_for(F.n, 1024)), dim3(kBlock), 0, L.st, (size_t)F.n, x, L.counter,
                     gate);
  int *err = &L.ctl->err;
  if (prof) L.prof->begin(L.st, &ev);
  if (F.lower)
    hipLaunchKernelGGL((k_trsv_sf<T, true>), dim3(nb), dim3(kBlock), 0, L.st, F.n, F.lev_rows, F.rp, F.ci, F.v, b, x,
                       kfuse, R, coef, L.counter, err, gate);
  else
    hipLaunchKernelGGL((k_trsv_sf<T, false>), dim3(nb), dim3(kBlock), 0, L.st, F.n, F.lev_rows, F.rp, F.ci, F.v, b,
                       x, kfuse, R, coef, L.counter, err, gate);
  if (prof) L.prof->end(L.st, pid, ev);
}

// ------------------------------------------------------------------ casts / fills
template <typename Tin, typename Tout>
__global__ void k_cast(size_t n, const Tin *in, Tout *out) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = (Tout)in[i];
}
template <typename Tin, typename Tout>
void launch_cast(hipStream_t st, size_t n, const Tin *in, Tout *out) {
  if (n == 0) return;
  hipLaunchKernelGGL((k_cast<Tin, Tout>), dim3(grid_for(n, 4096)), dim3(kBlock), 0, st, n, in, out);
}

template <typename T>
__global__ void k_fill(size_t n, T *x, T v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) x[i] = v;
}
template <typename T>
void launch_fill(hipStream_t st, size_t n, T *x, T v) {
  if (n == 0) return;
  hipLaunchKernelGGL((k_fill<T>), dim3(grid_for(n, 4096)), dim3(kBlock), 0, st, n, x, v);
}

// ------------------------------------------------------------------ instantiations
#define INST(T)                                                                                                      \
  template int launch_spmv<T>(const Launch &, const Mat<T> &, const T *, T *, int, const VList<T> &, int,            \
                              const VList<T> &, double *, const int *);                                              \
  template int launch_multidot<T, T>(const Launch &, int, int, const VList<T> &, const VList<T> &, double *,          \
                                     const int *);                                                                   \
  template void launch_trsv<T>(const Launch &, const Tri<T> &, const T *, T *, int, const VList<T> &, const double *, \
                               const int *);                                                                         \
  template void launch_fill<T>(hipStream_t, size_t, T *, T);
INST(double)
INST(float)
template int launch_multidot<float, double>(const Launch &, int, int, const VList<float> &, const VList<float> &,
                                            double *, const int *);
template void launch_cast<double, float>(hipStream_t, size_t, const double *, float *);
template void launch_cast<float, double>(hipStream_t, size_t, const float *, double *);
template void launch_cast<double, double>(hipStream_t, size_t, const double *, double *);

}  // namespace bnx
