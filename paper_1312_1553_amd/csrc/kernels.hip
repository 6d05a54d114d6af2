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
template <typename T, int MAXD, int RW>
__global__ __launch_bounds__(kBlock) void k_spmv_ell(int n, const int *__restrict__ eptr, const int *__restrict__ elen,
                                                     const int *__restrict__ ecol, const T *__restrict__ eval,
                                                     const T *__restrict__ x, T *__restrict__ y, int ndy, VList<T> ly,
                                                     int ndx, VList<T> lx, double *part, const int *gate) {
  if (gate && *gate) return;
  constexpr int NA = MAXD > 0 ? MAXD : 1;
  T acc[NA];
#pragma unroll
  for (int d = 0; d < NA; d++) acc[d] = T(0);
  // RW rows per thread together (stride apart), so their slice headers, entries and x gathers are in
  // flight at once: each row is a chain of three dependent loads
  const int stride = gridDim.x * kBlock;
  for (int row0 = blockIdx.x * kBlock + threadIdx.x; row0 < n; row0 += RW * stride) {
    int rr[RW], base[RW], len[RW];
#pragma unroll
    for (int u = 0; u < RW; u++) {
      rr[u] = row0 + u * stride;
      const int sl = (rr[u] < n ? rr[u] : row0) >> 6;
      base[u] = eptr[sl] + ((rr[u] < n ? rr[u] : row0) & 63);
      len[u] = rr[u] < n ? elen[sl] : 0;
    }
    int lmax = 0;
#pragma unroll
    for (int u = 0; u < RW; u++) lmax = len[u] > lmax ? len[u] : lmax;
    T s[RW];
#pragma unroll
    for (int u = 0; u < RW; u++) s[u] = T(0);
    // batches of 8 entries per row: all column and value loads issued before the x gathers
    for (int e0 = 0; e0 < lmax; e0 += 8) {
      int cc[RW][8];
      T vv[RW][8];
#pragma unroll
      for (int u = 0; u < RW; u++)
#pragma unroll
        for (int q = 0; q < 8; q++) {
          const bool ok = e0 + q < len[u];
          cc[u][q] = ok ? ecol[base[u] + 64 * (e0 + q)] : row0;
          vv[u][q] = ok ? eval[base[u] + 64 * (e0 + q)] : T(0);
        }
      T xx[RW][8];
#pragma unroll
      for (int u = 0; u < RW; u++)
#pragma unroll
        for (int q = 0; q < 8; q++) xx[u][q] = x[cc[u][q]];
#pragma unroll
      for (int u = 0; u < RW; u++)
#pragma unroll
        for (int q = 0; q < 8; q++) s[u] += vv[u][q] * xx[u][q];
    }
#pragma unroll
    for (int u = 0; u < RW; u++) {
      const int row = rr[u];
      if (row >= n) continue;
      y[row] = s[u];
      if (MAXD > 0) {
        const T xr = x[row];
#pragma unroll
        for (int d = 0; d < NA; d++) {
          if (d < ndy) acc[d] += s[u] * ly.p[d][row];
          else if (d < ndy + ndx) acc[d] += xr * lx.p[d - ndy][row];
        }
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
#define BNX_ELL(MD, RW)                                                                                        \
  hipLaunchKernelGGL((k_spmv_ell<T, MD, RW>), dim3(nb), dim3(kBlock), 0, L.st, A.n, A.ell_ptr, A.ell_len, A.ell_col, \
                     A.ell_val, x, y, ndy, ly, ndx, lx, part, gate)
    // two rows per thread for short rows (100^3 grid: fp32 17.2 -> 15.0 us, fp64 22.1 -> 21.0 us); long rows
    // (27-point elasticity, ~80 entries) already keep enough loads in flight, and two cost registers
    const bool two = A.group <= 16;
    if (nd == 0) {
      if (two) BNX_ELL(0, 2);
      else BNX_ELL(0, 1);
    } else if (nd <= 6) {
      if (two) BNX_ELL(6, 2);
      else BNX_ELL(6, 1);
    } else {
      if (two) BNX_ELL(72, 2);
      else BNX_ELL(72, 1);
    }
#undef BNX_ELL
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
  else if (D <= 24)  // the DACG dots of up to 11 deflated vectors (2 nq + 1) without the registers of 48
    hipLaunchKernelGGL((k_multidot<T, Acc, 24>), dim3(nb), dim3(kBlock), 0, L.st, n, D, X, Y, part, gate);
  else if (D <= 48)
    hipLaunchKernelGGL((k_multidot<T, Acc, 48>), dim3(nb), dim3(kBlock), 0, L.st, n, D, X, Y, part, gate);
  else
    hipLaunchKernelGGL((k_multidot<T, Acc, kMaxVec>), dim3(nb), dim3(kBlock), 0, L.st, n, D, X, Y, part, gate);
  return nb;
}

// Dots of one or two vectors A_a (a < NAV) with a list V (nv vectors), and of A_0 with A_1 (ab = 1):
//   part[a*nv + d] = sum_i A_a[i] V_d[i],   part[NAV*nv] = sum_i A_0[i] A_1[i]
// Every vector is read once per element (the generic multi-dot reads a vector once per dot it appears in).
// RW rows per thread (a grid stride apart) have their loads in flight together; each accumulator still adds
// the rows in grid-stride order, so the partials do not depend on RW.
template <typename T, typename Acc, int NAV, int MAXV, int RW>
__global__ __launch_bounds__(kBlock) void k_mdot_list(int n, const T *__restrict__ A0, const T *__restrict__ A1, int nv,
                                                      VList<T> V, int ab, double *part, const int *gate) {
  if (gate && *gate) return;
  constexpr int NA = NAV * MAXV + 1;
  Acc acc[NA];
#pragma unroll
  for (int j = 0; j < NA; j++) acc[j] = Acc(0);
  const int stride = gridDim.x * kBlock;
  for (int i0 = blockIdx.x * kBlock + threadIdx.x; i0 < n; i0 += RW * stride) {
    Acc a0[RW], a1[RW], vv[RW][MAXV];
#pragma unroll
    for (int u = 0; u < RW; u++) {
      const int i = i0 + u * stride < n ? i0 + u * stride : i0;
      a0[u] = (Acc)A0[i];
      a1[u] = NAV > 1 ? (Acc)A1[i] : Acc(0);
#pragma unroll
      for (int d = 0; d < MAXV; d++) vv[u][d] = d < nv ? (Acc)V.p[d][i] : Acc(0);
    }
#pragma unroll
    for (int u = 0; u < RW; u++) {
      if (i0 + u * stride >= n) break;
#pragma unroll
      for (int d = 0; d < MAXV; d++)
        if (d < nv) {
          acc[d] += a0[u] * vv[u][d];
          if (NAV > 1) acc[MAXV * (NAV - 1) + d] += a1[u] * vv[u][d];
        }
      if (NAV > 1) acc[NAV * MAXV] += a0[u] * a1[u];
    }
  }
  // slot j < NAV*MAXV holds A_{j / MAXV}^T V_{j % MAXV}; slot NAV*MAXV holds A_0^T A_1
  auto out_of = [&](int j) {
    if (j < NAV * MAXV) return (j % MAXV) < nv ? (j / MAXV) * nv + (j % MAXV) : -1;
    return (NAV > 1 && ab) ? NAV * nv : -1;
  };
  __shared__ double red[kBlock / 64][NA];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < NA; j++)
    if (out_of(j) >= 0) {
      const Acc sum = wave_sum(acc[j]);
      if (lane == 0) red[w][j] = (double)sum;
    }
  __syncthreads();
  for (int j = threadIdx.x; j < NA; j += kBlock) {
    const int out = out_of(j);
    if (out >= 0) {
      double sum = 0.0;
#pragma unroll
      for (int ww = 0; ww < kBlock / 64; ww++) sum += red[ww][j];
      part[(size_t)out * gridDim.x + blockIdx.x] = sum;
    }
  }
}

template <typename T, typename Acc>
int launch_mdot_list(const Launch &L, int n, int na, const T *A0, const T *A1, int nv, const VList<T> &V, int ab,
                     double *part, const int *gate) {
  const int nb = grid_for((size_t)n, L.nb);
  // two rows per thread while their loads fit in registers without lowering the occupancy the grid needs
  // (four waves per SIMD): up to 64 bytes of V per row (fp64 nv <= 8: 10.8 -> 9.5 us at nv <= 4; fp32 nv <= 12:
  // 16.5 -> 12.6 us); more (fp64 nv <= 12 took 178 VGPRs) gains nothing
#define BNX_MDL(NAV, MV)                                                                                          \
  hipLaunchKernelGGL((k_mdot_list<T, Acc, NAV, MV, ((MV) * sizeof(Acc) <= 64 ? 2 : 1)>), dim3(nb), dim3(kBlock), 0, \
                     L.st, n, A0, A1, nv, V, ab, part, gate)
  if (na == 1) {
    if (nv <= 8) BNX_MDL(1, 8);
    else if (nv <= 24) BNX_MDL(1, 24);
    else BNX_MDL(1, kMaxQ + kMaxK + 1);
  } else {
    if (nv <= 4) BNX_MDL(2, 4);
    else if (nv <= 8) BNX_MDL(2, 8);
    else if (nv <= 12) BNX_MDL(2, 12);
    else BNX_MDL(2, kMaxQ);
  }
#undef BNX_MDL
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

// right-hand side of row i of the system being solved: rhs_value, then the transform of a
// level-compressed system (its substituted rows' right-hand sides, weighted)
template <typename T>
__device__ __forceinline__ T rhs_sys(int i, const T *b, int kfuse, const VList<T> &R, const double *coef,
                                     const RhsT<T> &M) {
  T s = rhs_value(i, b, kfuse, R, coef);
  if (M.mp)
    for (int t = M.mp[i]; t < M.mp[i + 1]; t++) s -= M.mv[t] * rhs_value(M.mj[t], b, kfuse, R, coef);
  return s;
}

// One dependency level, one thread per row.  lower: x_i = (b_i - sum_{e<diag} L_e x_c)/L_diag (diag last);
// upper (rows of L^T): x_i = (b_i - sum_{e>diag} Lt_e x_c)/Lt_diag (diag first).
template <typename T, bool LOWER>
__global__ __launch_bounds__(kBlock) void k_trsv_level(int r0, int r1, const int *__restrict__ rows,
                                                       const int *__restrict__ rp, const int *__restrict__ ci,
                                                       const T *__restrict__ v, const T *__restrict__ b, T *x,
                                                       int kfuse, VList<T> R, const double *coef, RhsT<T> M,
                                                       const int *gate) {
  if (gate && *gate) return;
  int pos = r0 + blockIdx.x * kBlock + threadIdx.x;
  if (pos >= r1) return;
  const int i = rows[pos];
  T s = rhs_sys(i, b, kfuse, R, coef, M);
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
// Block solve: compute waves per workgroup per precision, importer waves, the rest publish (measured on the
// 100^3 grid's schedules, fp64 blocks of about 4k rows and fp32 about 8k: 4 to 12 compute waves, 1 to 4
// importers); s_wakeup of the workgroup after a round that stored values; s_sleep of a publisher poll.
#ifndef BNX_TRSV_WC64
#define BNX_TRSV_WC64 6
#endif
#ifndef BNX_TRSV_WC32
#define BNX_TRSV_WC32 8
#endif
#ifndef BNX_TRSV_WAKE
#define BNX_TRSV_WAKE 0
#endif
#ifndef BNX_TRSV_WI
#define BNX_TRSV_WI 3
#endif
#ifndef BNX_TRSV_KC32
#define BNX_TRSV_KC32 8
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
                                                    const double *coef, RhsT<T> M, int *counter, int *err,
                                                    const int *gate) {
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
      T s = rhs_sys(i, b, kfuse, R, coef, M);
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

template <typename T, int NR>
struct RowPre {
  int cnt;
  T d;
  int rr[NR];
  T vv[NR];
};

// Row data of rank k: rank-indexed loads only, none conditional (the caller
// passes a valid rank for lanes without a row), so the compiler can count the
// loads in flight exactly and wait only for the ones it needs.
template <typename T, int NR>
__device__ __forceinline__ void row_fetch(const DevBlk<T> &F, int k, RowPre<T, NR> &P) {
  const int np = F.npad;
  P.cnt = F.cnt[k];
  P.d = F.diag[k];  // reciprocal of the diagonal
#pragma unroll
  for (int q = 0; q < NR; q++) {
    P.rr[q] = F.ref4[(size_t)q * np + k];
    P.vv[q] = F.val4[(size_t)q * np + k];
  }
}

// LDS-staged sync-free solve.  One 1024-thread workgroup per block of the
// schedule (blocks taken in order from a ticket counter; the order is
// topological, so a block only waits on blocks that started before it).  Every
// value a block reads lives in its LDS: its own rows at their local rank and
// the values it imports from earlier blocks behind them.
//  * WC compute waves walk the block's 64-row slices in order (wave w takes
//    slices w, w+WC, ...).  A lane polls its row's dependencies in LDS, and
//    writes the result to LDS only, so compute waves never touch global memory
//    for the dependency chain.
//  * WP publisher waves copy finished values to the solution x in global
//    memory (device-scope stores: other blocks import from there).
//  * WI importer waves poll x for the block's imports, in order of first use,
//    and copy them into LDS.
// Every dependency of a row has a lower rank or is an import, so the lowest
// unfinished row can always proceed.  Waits are bounded: on overflow the value
// becomes NaN and *err is set.
// The launch also does what a separate preparation pass would: it gathers the
// right-hand side of its rows into LDS (b_i minus the fused first loop of Alg. 1,
// sum_t coef[t] R_t[i], then the transform M of a level-compressed system), and
// it resets the other half of the export buffer and its ticket counter for the
// next launch of this precision (also when the launch is gated off).
template <typename T, int CAP, bool LONG, int NR>
__global__ __launch_bounds__(1024) void k_trsv_blk(DevBlk<T> F, const T *__restrict__ b, int kfuse, VList<T> R,
                                                    const double *coef, RhsT<T> M, T *x, T *xe_pair, int nexp_half,
                                                    int par, int *cnt_pair, int *err, const int *gate) {
  using U = typename Sentinel<T>::U;
  {
    U *xo = reinterpret_cast<U *>(xe_pair) + (size_t)(1 - par) * nexp_half;
    for (int i = blockIdx.x * 1024 + threadIdx.x; i < nexp_half; i += gridDim.x * 1024) xo[i] = Sentinel<T>::bits;
    if (blockIdx.x == 0 && threadIdx.x == 0) cnt_pair[1 - par] = 0;
  }
  if (gate && *gate) return;
  T *xe = xe_pair + (size_t)par * nexp_half;
  constexpr int WC = sizeof(T) == 8 ? BNX_TRSV_WC64 : BNX_TRSV_WC32, WI = BNX_TRSV_WI;
  constexpr int WP = 16 - WC - WI;
  static_assert(WP >= 1 && WI >= 1, "wave roles");
  __shared__ U xs[CAP];
  __shared__ int blk_s;
  if (threadIdx.x == 0) blk_s = atomicAdd(cnt_pair + par, 1);
  __syncthreads();
  const int blk = blk_s;
  if (blk >= F.nblocks) return;
  const int k0 = F.bptr[blk], nrow = F.brows[blk];
  const int i0 = F.iptr[blk], nimp = F.iptr[blk + 1] - i0;
  // LDS: rows [0, nrow), imports [nrow, nrow + nimp), the zero slot, the right-hand side of the rows, then
  // a dump slot that lanes past the last row write to
  const int rb = nrow + nimp + 1;
  for (int i = threadIdx.x; i <= nrow + nimp; i += 1024) xs[i] = i < nrow + nimp ? Sentinel<T>::bits : U(0);
  // right-hand side of the block's ranks (0 for a virtual row), PU ranks per thread whose loads are
  // in flight together: the row and transform indices first, then every value they name
  constexpr int PU = 4;
  for (int t0 = threadIdx.x; t0 < nrow; t0 += PU * 1024) {
    int ii[PU], kk[PU];
    T v[PU];
#pragma unroll
    for (int u = 0; u < PU; u++) {
      const int t = t0 + u * 1024;
      kk[u] = k0 + (t < nrow ? t : 0);
      ii[u] = t < nrow ? F.perm[kk[u]] : -1;
    }
#pragma unroll
    for (int u = 0; u < PU; u++) v[u] = ii[u] >= 0 ? b[ii[u]] : T(0);
    for (int q = 0; q < kfuse; q++) {  // w = g - R a (first loop of Alg. 1)
      const T cq = (T)coef[q];
      const T *Rq = R.p[q];
#pragma unroll
      for (int u = 0; u < PU; u++)
        if (ii[u] >= 0) v[u] -= cq * Rq[ii[u]];
    }
    // transform of a level-compressed system, EU slots at a time: the slot indices are rank-indexed and
    // load beside the row ids (a virtual or padding rank names no row: -1), then every value they name
    constexpr int EU = 4;
    for (int e0 = 0; e0 < F.mw; e0 += EU) {
      int jj[EU][PU], ww[EU][PU];
      T rj[EU][PU];
#pragma unroll
      for (int ee = 0; ee < EU; ee++)
#pragma unroll
        for (int u = 0; u < PU; u++) {
          const bool in = e0 + ee < F.mw;
          const size_t at = (size_t)(in ? e0 + ee : 0) * F.npad + kk[u];
          jj[ee][u] = in ? F.mjr[at] : -1;
          ww[ee][u] = in ? F.mtr[at] : 0;
        }
#pragma unroll
      for (int ee = 0; ee < EU; ee++)
#pragma unroll
        for (int u = 0; u < PU; u++) rj[ee][u] = jj[ee][u] >= 0 ? b[jj[ee][u]] : T(0);
      for (int q = 0; q < kfuse; q++) {
        const T cq = (T)coef[q];
        const T *Rq = R.p[q];
#pragma unroll
        for (int ee = 0; ee < EU; ee++)
#pragma unroll
          for (int u = 0; u < PU; u++)
            if (jj[ee][u] >= 0) rj[ee][u] -= cq * Rq[jj[ee][u]];
      }
#pragma unroll
      for (int ee = 0; ee < EU; ee++)
#pragma unroll
        for (int u = 0; u < PU; u++)
          if (jj[ee][u] >= 0) v[u] -= M.mv[ww[ee][u]] * rj[ee][u];
    }
#pragma unroll
    for (int u = 0; u < PU; u++) {
      const int t = t0 + u * 1024;
      if (t < nrow) xs[rb + t] = to_bits<T>(v[u]);
    }
  }
  __syncthreads();
  U *xeu = reinterpret_cast<U *>(xe);
  const int nsl = (nrow + 63) >> 6;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;

  if (wave >= WC + WP) {  // importer: two imports per lane in flight, the next two rows prefetched
    const int step = WI * 128;
    int base = (wave - WC - WP) * 128;
    int r0 = base + lane < nimp ? F.isrc[i0 + base + lane] : -1;
    int r1 = base + 64 + lane < nimp ? F.isrc[i0 + base + 64 + lane] : -1;
    for (; base < nimp; base += step) {
      const int e0 = base + lane, e1 = base + 64 + lane;
      const int n0 = base + step + lane < nimp ? F.isrc[i0 + base + step + lane] : -1;
      const int n1 = base + step + 64 + lane < nimp ? F.isrc[i0 + base + step + 64 + lane] : -1;
      bool p0 = r0 >= 0, p1 = r1 >= 0;
      int spins = 0;
      while (__builtin_amdgcn_ballot_w64(p0 || p1) != 0ull) {
        if (p0 || p1) {
          U u0 = p0 ? __hip_atomic_load(&xeu[r0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : Sentinel<T>::bits;
          U u1 = p1 ? __hip_atomic_load(&xeu[r1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : Sentinel<T>::bits;
          if (++spins > kSpinLimit) {  // bounded wait: pending imports become NaN
            const U nan = to_bits<T>(T(__builtin_nan("")));
            if (u0 == Sentinel<T>::bits) u0 = nan;
            if (u1 == Sentinel<T>::bits) u1 = nan;
            atomicOr(err, 1);
          }
          if (p0 && u0 != Sentinel<T>::bits) {
            __hip_atomic_store(&xs[nrow + e0], u0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            p0 = false;
          }
          if (p1 && u1 != Sentinel<T>::bits) {
            __hip_atomic_store(&xs[nrow + e1], u1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            p1 = false;
          }
        }
        if (BNX_TRSV_WAKE) __asm__ volatile("s_wakeup");
      }
      r0 = n0;
      r1 = n1;
    }
  } else if (wave >= WC) {
    // publisher: the block's exports, PG per lane in flight, each value goes out as soon as it is in LDS
    constexpr int PG = 4;
    const int e0 = F.eptr[blk], nex = F.eptr[blk + 1] - e0;
    const int p = wave - WC, gstep = WP * 64 * PG;
    // group j of publisher p: exports e0 + p*64*PG + j*gstep + g*64 + lane, g < PG
    auto group_slots = [&](int j, int (&r)[PG]) {
#pragma unroll
      for (int g = 0; g < PG; g++) {
        const int e = p * 64 * PG + j * gstep + g * 64 + lane;
        r[g] = e < nex ? F.erank[e0 + e] : -1;
      }
    };
    int cur[PG], nxt[PG];
    group_slots(0, cur);
    for (int j = 0; p * 64 * PG + j * gstep < nex; j++) {
      group_slots(j + 1, nxt);
      unsigned pend = 0;
#pragma unroll
      for (int g = 0; g < PG; g++) pend |= (cur[g] >= 0 ? 1u : 0u) << g;
      int spins = 0;
      while (__builtin_amdgcn_ballot_w64(pend != 0u) != 0ull) {
        if (pend) {
          U u[PG];
#pragma unroll
          for (int g = 0; g < PG; g++)
            u[g] = (pend >> g & 1u) ? __hip_atomic_load(&xs[cur[g]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)
                                    : Sentinel<T>::bits;
          const bool over = ++spins > kSpinLimit;
          if (over) atomicOr(err, 1);
#pragma unroll
          for (int g = 0; g < PG; g++)
            if (pend >> g & 1u) {
              U v = u[g];
              if (v == Sentinel<T>::bits && over) v = to_bits<T>(T(__builtin_nan("")));
              if (v != Sentinel<T>::bits) {
                const int e = p * 64 * PG + j * gstep + g * 64 + lane;
                __hip_atomic_store(&xeu[e0 + e], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                pend &= ~(1u << g);
              }
            }
        }
        if (BNX_TRSV_PUBSLEEP > 0) __builtin_amdgcn_s_sleep(BNX_TRSV_PUBSLEEP);
      }
#pragma unroll
      for (int g = 0; g < PG; g++) cur[g] = nxt[g];
    }
  } else {
  // compute: row data of the next three slices in flight while one is solved;
  // the four buffers rotate statically (no register copies, which would wait on
  // the loads in flight)
  auto fetch = [&](int sl, RowPre<T, NR> &P) {
    const int t = (sl << 6) + lane;
    row_fetch<T, NR>(F, (sl < nsl && t < nrow) ? k0 + t : k0, P);
  };
  // The polling loop runs until no lane of the wave is pending (a ballot), so a
  // row's store sits inside the iteration in which it finishes: code after a
  // divergent loop exit would only run once the whole wave has left the loop,
  // and rows of one slice may depend on each other.
  auto solve_slice = [&](const RowPre<T, NR> &cur, int sl) {
    const int t = (sl << 6) + lane;
    bool fin = t >= nrow;
    const T s0 = fin ? T(0) : from_bits<T>(xs[rb + t]);
    const int gsl = (k0 >> 6) + sl;
    // lane 0 always holds a row of the slice; its flag tells whether any row is long (schedules
    // without long rows run the instantiation that has no general path)
    if (!LONG || (__builtin_amdgcn_readfirstlane(cur.cnt) & kLongSlice) == 0) {
      // every row of the slice has at most NR dependencies (unused ones read the zero slot).  Each
      // round every lane reads its NR values (finished lanes too: their addresses are valid) and stores
      // one word: its value once all NR are in, else the sentinel again.  A finished row rewrites the
      // same bits (its inputs no longer change), and a lane past the block writes a dump slot behind
      // the right-hand side.  The sentinel test looks only at the high 32 bits of a double: they are
      // those of a signalling NaN, which no arithmetic result, and hence no stored value, has.  Per
      // round that leaves two wave-uniform exits and no exec-mask work: the 16 waves of a workgroup
      // share the CU's scalar unit.
      constexpr unsigned SH = (unsigned)(Sentinel<T>::bits >> (8 * sizeof(U) - 32));
      const int dst = t < nrow ? t : rb + nrow;
      unsigned pend = fin ? 0u : 1u;
      int left = kSpinLimit;
      for (;;) {
        U u[NR];
#pragma unroll
        for (int q = 0; q < NR; q++)
          u[q] = __hip_atomic_load(&xs[-cur.rr[q] - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        unsigned m = 0xffffffffu;  // zero iff a dependency still holds the sentinel
        T acc = s0;
#pragma unroll
        for (int q = 0; q < NR; q++) {
          const unsigned hi = (unsigned)(u[q] >> (8 * sizeof(U) - 32));
          m = min(m, hi ^ SH);
          acc -= cur.vv[q] * from_bits<T>(u[q]);
        }
        const U w = m != 0u ? to_bits<T>(acc * cur.d) : Sentinel<T>::bits;
        __hip_atomic_store(&xs[dst], w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        pend = m != 0u ? 0u : pend;
        if (__builtin_amdgcn_ballot_w64(pend != 0u) == 0ull) break;
        if (--left == 0) break;
      }
      if (pend) {  // the bounded wait ran out
        __hip_atomic_store(&xs[t], to_bits<T>(T(__builtin_nan(""))), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        atomicOr(err, 1);
      }
      return;
    }
    if constexpr (LONG) {
    // general path: the first NR dependencies (unused slots read the zero slot), then the
    // rest from the ELL slices in chunks of KC independent loads, consumed in order
    constexpr int KC = sizeof(T) == 8 ? 4 : BNX_TRSV_KC32;
    const int nlong = cur.cnt & ~kLongSlice;
    const int esp = F.slice_ptr[gsl] + lane;
    int cr[KC];
    T cv[KC];
    int e = NR;                // next ELL entry to load
    int cpos = KC, cend = KC;  // consumed / valid entries of the chunk in registers
    auto load_chunk = [&]() {
      const int m = nlong - e < KC ? nlong - e : KC;
#pragma unroll
      for (int q = 0; q < KC; q++) {
        const int at = esp + 64 * (e + q - NR);
        cr[q] = q < m ? F.ref[at] : -1;
        cv[q] = q < m ? F.val[at] : T(0);
      }
      e += m;
      cpos = 0;
      cend = m;
    };
    if (!fin && nlong > NR) load_chunk();  // in flight while the first NR are polled
    bool head = false;                     // the first NR are consumed
    T s = s0;
    int spins = 0;
    while (__builtin_amdgcn_ballot_w64(!fin) != 0ull) {
      if (!fin) {
        if (!head) {
          U lv[NR];
#pragma unroll
          for (int q = 0; q < NR; q++)
            lv[q] = __hip_atomic_load(&xs[-cur.rr[q] - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          bool ok = true;
#pragma unroll
          for (int q = 0; q < NR; q++) ok = ok && lv[q] != Sentinel<T>::bits;
          if (ok) {
#pragma unroll
            for (int q = 0; q < NR; q++) s -= cur.vv[q] * from_bits<T>(lv[q]);
            head = true;
          }
        }
        if (head) {
          for (;;) {
            if (cpos == cend) {
              if (e >= nlong) break;
              load_chunk();
            }
            U u[KC];
#pragma unroll
            for (int q = 0; q < KC; q++)
              u[q] = (q >= cpos && q < cend)
                         ? __hip_atomic_load(&xs[-cr[q] - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)
                         : Sentinel<T>::bits;
            int c = cpos;
#pragma unroll
            for (int q = 0; q < KC; q++)  // the ready prefix, in entry order
              if (q == c && q < cend && u[q] != Sentinel<T>::bits) {
                s -= cv[q] * from_bits<T>(u[q]);
                c++;
              }
            cpos = c;
            if (cpos < cend) break;  // blocked: poll again next round
          }
          if (cpos == cend && e >= nlong) {
            __hip_atomic_store(&xs[t], to_bits<T>(s * cur.d), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            fin = true;
          }
        }
        if (!fin && ++spins > kSpinLimit) {
          __hip_atomic_store(&xs[t], to_bits<T>(T(__builtin_nan(""))), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WORKGROUP);
          atomicOr(err, 1);
          fin = true;
        }
      }
    }
    }
  };
  RowPre<T, NR> A, B, C, D;
  fetch(wave, A);
  fetch(wave + WC, B);
  fetch(wave + 2 * WC, C);
  for (int sl = wave; sl < nsl; sl += 4 * WC) {
    fetch(sl + 3 * WC, D);
    solve_slice(A, sl);
    if (sl + WC >= nsl) break;
    fetch(sl + 4 * WC, A);
    solve_slice(B, sl + WC);
    if (sl + 2 * WC >= nsl) break;
    fetch(sl + 5 * WC, B);
    solve_slice(C, sl + 2 * WC);
    if (sl + 3 * WC >= nsl) break;
    fetch(sl + 6 * WC, C);
    solve_slice(D, sl + 3 * WC);
  }
  }
  // every row of the block is in LDS: write the solution once, in row order
  __syncthreads();
  for (int t = threadIdx.x; t < nrow; t += 1024) {
    const int r = F.orow[k0 + t];  // virtual rows (-1) come last and are not written
    if (r >= 0) x[r] = from_bits<T>(xs[F.oslot[k0 + t]]);
  }
}

// Latency probes: a chain of `hops` dependent hand-overs, timed as one launch.
// k_probe_lds: one workgroup; hop h is taken by wave h mod 16, which waits until
// the LDS flag holds h-1 and then writes h (the same hand-over as a dependency
// between two compute waves of the block solve).  k_probe_global: one
// workgroup per hop in ticket order; each waits for its predecessor's
// device-scope flag in global memory and then sets its own (the hand-over
// between two blocks).  Waits are bounded; on overflow *err is set.
__global__ __launch_bounds__(1024) void k_probe_lds(int hops, int *err) {
  __shared__ int flag;
  if (threadIdx.x == 0) flag = -1;
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int h = wave; h < hops; h += 16) {
    int spins = 0;
    while (__hip_atomic_load(&flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != h - 1) {
      if (++spins > kSpinLimit) {
        if (lane == 0) atomicOr(err, 1);
        break;
      }
    }
    if (lane == 0) __hip_atomic_store(&flag, h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
}

__global__ __launch_bounds__(64) void k_probe_global(int *flags, int *counter, int *err) {
  __shared__ int ticket;
  if (threadIdx.x == 0) ticket = atomicAdd(counter, 1);
  __syncthreads();
  if (threadIdx.x != 0) return;
  const int me = ticket;
  if (me > 0) {
    int spins = 0;
    while (__hip_atomic_load(&flags[me - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
      if (++spins > kSpinLimit) {
        atomicOr(err, 1);
        break;
      }
  }
  __hip_atomic_store(&flags[me], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

void launch_probe(hipStream_t st, int kind, int hops, int *flags, int *counter, int *err) {
  if (kind == 0) {
    hipLaunchKernelGGL(k_probe_lds, dim3(1), dim3(1024), 0, st, hops, err);
  } else {
    launch_fill<int>(st, (size_t)hops, flags, 0);
    launch_fill<int>(st, 1, counter, 0);
    hipLaunchKernelGGL(k_probe_global, dim3(hops), dim3(64), 0, st, flags, counter, err);
  }
}

template <typename T, int CAP>
static void launch_blk(const Launch &L, const Tri<T> &F, const T *b, int kfuse, const VList<T> &R,
                       const double *coef, T *x, int par, const int *gate) {
#define BNX_BLK(LONG, NR)                                                                                         \
  hipLaunchKernelGGL((k_trsv_blk<T, CAP, LONG, NR>), dim3(F.blk.nblocks), dim3(1024), 0, L.st, F.blk, b, kfuse,  \
                     R, coef, F.M, x, F.blk_exp, F.blk_nexp, par, F.blk_cnt, &L.ctl->err, gate)
  // three-slot schedules (no row longer than three), level-compressed systems (kNRC slots)
  // and wide split schedules (kNRW slots, float only: eight double slots spill registers)
  // have no row beyond their slots and need no general path
  if (F.blk.nr == 3) {
    BNX_BLK(false, 3);
  } else if (F.blk.nr == kNRC) {
    BNX_BLK(false, kNRC);
  } else if (sizeof(T) == 4 && F.blk.nr == kNRW) {
    if constexpr (sizeof(T) == 4) BNX_BLK(false, kNRW);
  } else if (F.blk.ell > 0) {
    BNX_BLK(true, kNR);
  } else {
    BNX_BLK(false, kNR);
  }
#undef BNX_BLK
}

template <typename T>
void launch_blk_reset(hipStream_t st, T *xe_pair, int nexp_half, int *cnt_pair) {
  const size_t m = 2 * (size_t)nexp_half;
  hipLaunchKernelGGL((k_sentinel<T>), dim3(grid_for(m > 0 ? m : 1, 1024)), dim3(kBlock), 0, st, m, xe_pair, cnt_pair,
                     nullptr);
  hipLaunchKernelGGL((k_sentinel<T>), dim3(1), dim3(kBlock), 0, st, (size_t)0, xe_pair, cnt_pair + 1, nullptr);
}

template <typename T>
void launch_trsv(const Launch &L, const Tri<T> &F, const T *b, T *x, int kfuse, const VList<T> &R,
                 const double *coef, const int *gate) {
  if (L.trsv_mode == 0 && F.blk.nblocks > 0) {
    const bool prof0 = L.prof && L.prof->on;
    hipEvent_t ev0 = nullptr;
    const int par = (int)((*F.blk_seq)++ & 1);
    if (prof0) L.prof->begin(L.st, &ev0);
    if constexpr (sizeof(T) == 8) launch_blk<T, kLdsCap64>(L, F, b, kfuse, R, coef, x, par, gate);
    else launch_blk<T, kLdsCap32>(L, F, b, kfuse, R, coef, x, par, gate);
    if (prof0) L.prof->end(L.st, (F.lower ? 2 : 4) + (sizeof(T) == 8 ? 0 : 1), ev0);
    return;
  }
  const bool prof = L.prof && L.prof->on;
  const int pid = (F.lower ? 2 : 4) + (sizeof(T) == 8 ? 0 : 1);
  hipEvent_t ev = nullptr;
  if (L.trsv_mode == 1) {  // one launch per dependency level
    if (prof) L.prof->begin(L.st, &ev);
    for (int l = 0; l < F.nlev; l++) {
      int r0 = (*F.lev_ptr)[l], r1 = (*F.lev_ptr)[l + 1];
      int nb = (r1 - r0 + kBlock - 1) / kBlock;
      if (F.lower)
        hipLaunchKernelGGL((k_trsv_level<T, true>), dim3(nb), dim3(kBlock), 0, L.st, r0, r1, F.lev_rows, F.rp, F.ci,
                           F.v, b, x, kfuse, R, coef, F.M, gate);
      else
        hipLaunchKernelGGL((k_trsv_level<T, false>), dim3(nb), dim3(kBlock), 0, L.st, r0, r1, F.lev_rows, F.rp,
                           F.ci, F.v, b, x, kfuse, R, coef, F.M, gate);
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
                       kfuse, R, coef, F.M, L.counter, err, gate);
  else
    hipLaunchKernelGGL((k_trsv_sf<T, false>), dim3(nb), dim3(kBlock), 0, L.st, F.n, F.lev_rows, F.rp, F.ci, F.v, b,
                       x, kfuse, R, coef, F.M, L.counter, err, gate);
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
  template int launch_mdot_list<T, T>(const Launch &, int, int, const T *, const T *, int, const VList<T> &, int,      \
                                      double *, const int *);                                                        \
  template void launch_trsv<T>(const Launch &, const Tri<T> &, const T *, T *, int, const VList<T> &, const double *, \
                               const int *);                                                                         \
  template void launch_fill<T>(hipStream_t, size_t, T *, T);                                                \
  template void launch_blk_reset<T>(hipStream_t, T *, int, int *);
INST(double)
INST(float)
template int launch_multidot<float, double>(const Launch &, int, int, const VList<float> &, const VList<float> &,
                                            double *, const int *);
template void launch_fill<int>(hipStream_t, size_t, int *, int);
template void launch_cast<double, float>(hipStream_t, size_t, const double *, float *);
template void launch_cast<float, double>(hipStream_t, size_t, const float *, double *);
template void launch_cast<double, double>(hipStream_t, size_t, const double *, double *);

}  // namespace bnx
