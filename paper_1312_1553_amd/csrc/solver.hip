// DACG-Newton driver (Alg. 2) and the C-ABI of the bnx library.
//
// One PCG iteration on the correction equation (Sec. 4.3, Sec. 3.2) is, on the
// device, with no host round trip:
//   trsv L  (rhs w = g - R a fused: first loop of Alg. 1)  ->  trsv L^T  ->
//   multi-dot (R^T c0, Q^T c0, g^T c0)  ->  control: second-loop coefficients,
//   CGS coefficients, rho, beta  ->  p = c0 - S(a+b) - Q z + beta p  ->
//   SpMV ap = A p with dots (p^T ap, p^T p, Q^T ap, Q^T p)  ->  control: gamma  ->
//   update s, g, t = A s with dots (||g||, eigen-residual terms, S^T g, Q^T g)  ->
//   eigen-residual pass  ->  control: exit tests (i)-(iv), first-loop coefficients.
// The two loops of Alg. 1 are evaluated in compact form: with sigma = S^T g and
// M[s][t] = s_s^T r_t, the first loop gives a_s = (sigma_s - sum_{t>s} a_t M[s][t])/alpha_s
// and, with rho_s = r_s^T c0, the second loop b_s = (rho_s - sum_{t<s} (a_t+b_t) M[t][s])/alpha_s;
// both equal the sequential recursions in exact arithmetic.  The CGS projection
// z = Q^T c uses Q^T c = Q^T c0 - (Q^T S)(a+b).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>

#include "../../include/bnx.h"
#include "fused.h"
#include "internal.h"

using namespace bnx;

#define HIPCHK(x)                                                                  \
  do {                                                                             \
    hipError_t e_ = (x);                                                           \
    if (e_ != hipSuccess) throw HipError(std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

namespace {

struct HipError {
  std::string msg;
  explicit HipError(std::string m) : msg(std::move(m)) {}
};
struct ApiError {
  bnx_status code;
  std::string msg;
};

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ============================================================== device helpers
// Convergence flag of an iteration, written straight into pinned host memory, where the host reads it
// (no copy and no event).
__device__ void post_flag(int *hflag, int v) {
  __hip_atomic_store(hflag, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  __threadfence_system();
}

// DEV: store with device-scope atomic stores, for a reduction fused into the same launch
template <typename T, int MAXD, bool DEV = false>
__device__ __forceinline__ void bpart(T (&acc)[MAXD], int nd, double *part) {
  __shared__ double red[4][MAXD];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int d = 0; d < MAXD; d++)
    if (d < nd) {
      T s = wsum(acc[d]);
      if (lane == 0) red[w][d] = (double)s;
    }
  __syncthreads();
  if (threadIdx.x < nd)
    store_partial(part + (size_t)threadIdx.x * gridDim.x + blockIdx.x,
                  red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x], DEV);
}

#define GRIDLOOP(i, n) for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += gridDim.x * blockDim.x)

// puts the empty mark into every slot of the fused-reduction area
__global__ void k_arm(unsigned long long *p, int cnt) { GRIDLOOP(i, cnt) p[i] = kEmptyMark; }

// The Gram quantities of the BFGS pairs that the serial recurrences of a control step read (M, the first
// k rows; alpha), copied into LDS by the whole block first: one thread then reads LDS, not global memory, in
// its dependent loops.  Ends with a barrier.
struct GramLds {
  double M[kMaxK * kMaxK], alpha[kMaxK], a[kMaxK];
};
__device__ __forceinline__ void stage_gram(const DevCtl *c, int k, GramLds &G) {
  for (int i = threadIdx.x; i < k * kMaxK; i += blockDim.x) G.M[i] = c->M[i];
  for (int i = threadIdx.x; i < k; i += blockDim.x) G.alpha[i] = c->alpha[i];
  __syncthreads();
}

// First loop of Alg. 1 in compact form: a_s for s = k-1..0 (sig and G in LDS).
__device__ void first_loop(DevCtl *c, int k, const double *sig, GramLds &G) {
  for (int s = k - 1; s >= 0; s--) {
    double v = sig[s];
    for (int t = s + 1; t < k; t++) v -= G.a[t] * G.M[s * kMaxK + t];
    G.a[s] = v / G.alpha[s];
    c->a[s] = G.a[s];
  }
}

// ============================================================== PCG kernels
// g = sgn * (r - Q (Q^T r)), s = 0, t = 0; dots: g^T g, S_t^T g (k), Q_c^T g (m)
template <typename T, int MAXD>
__global__ __launch_bounds__(kBlock) void k_pcg_init(int n, const DevCtl *c, double sgn, const T *r, int m, VList<T> Q,
                                                     int k, VList<T> S, T *g, T *s, T *t, double *part) {
  __shared__ T qr[kMaxQ];  // coefficients read once per workgroup
  for (int q = threadIdx.x; q < m; q += kBlock) qr[q] = (T)c->Qr[q];
  __syncthreads();
  T acc[MAXD];
#pragma unroll
  for (int d = 0; d < MAXD; d++) acc[d] = T(0);
  GRIDLOOP(i, n) {
    T v = r[i];
    for (int q = 0; q < m; q++) v -= qr[q] * Q.p[q][i];
    v *= (T)sgn;
    g[i] = v;
    s[i] = T(0);
    if (t) t[i] = T(0);
    acc[0] += v * v;
#pragma unroll
    for (int d = 1; d < MAXD; d++) {
      if (d <= k) acc[d] += S.p[d - 1][i] * v;
      else if (d <= k + m) acc[d] += Q.p[d - 1 - k][i] * v;
    }
  }
  bpart<T, MAXD>(acc, 1 + k + m, part);
}

// y = ap - theta p - Q zy;  s += gamma p;  g -= gamma y;  t += gamma ap
// dots: g^T g, [x^T (Au + t), x^T x with x = u + s], Q^T g (m), S^T g (k)
// RW rows a grid stride apart per pass have their loads in flight together (every sum still takes the rows
// in grid-stride order); the first MQ columns of Q stay in registers between y and the dots, so each is
// read once (Q's dots come before the BFGS ones so that their accumulators have compile-time slots).
template <typename T, int MAXD, int RW, int MQ>
__global__ __launch_bounds__(kBlock) void k_pcg_update(int n, const DevCtl *c, const T *ap, const T *p, int m,
                                                       VList<T> Q, int k, VList<T> S, const T *u, const T *Au, T *s,
                                                       T *g, T *t, double *part) {
  if (c->done) return;
  const T theta = (T)c->theta, gamma = (T)c->gamma;
  const int eig = c->eigtest;
  __shared__ T zy[kMaxQ];  // coefficients read once per workgroup
  for (int q = threadIdx.x; q < m; q += kBlock) zy[q] = (T)c->zy[q];
  __syncthreads();
  T acc[MAXD];
#pragma unroll
  for (int d = 0; d < MAXD; d++) acc[d] = T(0);
  const int stride = gridDim.x * blockDim.x;
  for (int i0 = blockIdx.x * blockDim.x + threadIdx.x; i0 < n; i0 += RW * stride) {
    int ii[RW];
    bool live[RW];
#pragma unroll
    for (int r = 0; r < RW; r++) {
      live[r] = i0 + r * stride < n;
      ii[r] = live[r] ? i0 + r * stride : i0;
    }
    T y[RW], gi[RW], si[RW], api[RW];
    T qc[RW][MQ > 0 ? MQ : 1];
#pragma unroll
    for (int r = 0; r < RW; r++) {
      api[r] = ap[ii[r]];
      const T pi = p[ii[r]];
      y[r] = api[r] - theta * pi;
      si[r] = s[ii[r]] + gamma * pi;
      gi[r] = g[ii[r]];
    }
#pragma unroll
    for (int q = 0; q < MQ; q++)
      if (q < m) {
#pragma unroll
        for (int r = 0; r < RW; r++) {
          qc[r][q] = Q.p[q][ii[r]];
          y[r] -= zy[q] * qc[r][q];
        }
      }
    for (int q = MQ; q < m; q++) {
      const T *qv = Q.p[q];
#pragma unroll
      for (int r = 0; r < RW; r++) y[r] -= zy[q] * qv[ii[r]];
    }
#pragma unroll
    for (int r = 0; r < RW; r++) {
      if (!live[r]) break;
      const int i = ii[r];
      gi[r] = gi[r] - gamma * y[r];
      s[i] = si[r];
      g[i] = gi[r];
      acc[0] += gi[r] * gi[r];
      if (eig) {
        const T ti = t[i] + gamma * api[r];
        t[i] = ti;
        const T xi = u[i] + si[r];
        acc[1] += xi * (Au[i] + ti);
        acc[2] += xi * xi;
      }
#pragma unroll
      for (int d = 3; d < MAXD; d++) {
        if (d < 3 + m) acc[d] += (d - 3 < MQ ? qc[r][d - 3 < MQ ? d - 3 : 0] : Q.p[d - 3][i]) * gi[r];
        else if (d < 3 + m + k) acc[d] += S.p[d - 3 - m][i] * gi[r];
      }
    }
  }
  bpart<T, MAXD>(acc, 3 + k + m, part);
}

// sum_i (Au_i + t_i - q (u_i + s_i))^2
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pcg_eigres(int n, const DevCtl *c, const T *u, const T *Au, const T *s,
                                                       const T *t, double *part) {
  if (c->done || !c->eigtest) return;
  const T q = (T)c->q;
  T acc[1] = {T(0)};
  GRIDLOOP(i, n) {
    const T d = Au[i] + t[i] - q * (u[i] + s[i]);
    acc[0] += d * d;
  }
  bpart<T, 1>(acc, 1, part);
}

// p = c0 - sum_s e_s S_s - sum_q zQ_q Q_q + beta p    (beta = 0 on the first application)
// dots (when nd > 0): Q_q^T p (m), then (A Q_q)^T p (m): with them Q^T (A - theta I) p = (AQ)^T p - theta Q^T p
template <typename T, int MAXD>
__global__ __launch_bounds__(kBlock) void k_pcg_newp(int n, const DevCtl *c, const T *c0, int k, VList<T> S, int m,
                                                     VList<T> Q, T *p, int with_beta, int nd, VList<T> AQ,
                                                     double *part) {
  if (c->done) return;
  const T beta = (T)c->beta;
  __shared__ T es[kMaxK], zq[kMaxQ];  // coefficients read once per workgroup
  for (int t = threadIdx.x; t < k; t += kBlock) es[t] = (T)c->e[t];
  for (int q = threadIdx.x; q < m; q += kBlock) zq[q] = (T)c->zQ[q];
  __syncthreads();
  constexpr int NA = MAXD > 0 ? MAXD : 1;
  // Q columns kept in registers between the combination and the dots, as many as leave the four waves per
  // SIMD the grid needs (MAXD = 2 m_max when dots are asked; six of twelve: 118 VGPRs in fp64)
  constexpr int MQ = MAXD == 8 ? 4 : (MAXD == 24 ? 6 : 0);
  T acc[NA];
#pragma unroll
  for (int d = 0; d < NA; d++) acc[d] = T(0);
  // two rows a grid stride apart per pass (loads of both in flight together); every sum still takes the
  // rows in grid-stride order
  const int stride = gridDim.x * blockDim.x;
  for (int i0 = blockIdx.x * blockDim.x + threadIdx.x; i0 < n; i0 += 2 * stride) {
    const bool two = i0 + stride < n;
    const int i1 = two ? i0 + stride : i0;
    T v0 = c0[i0], v1 = c0[i1];
    for (int s = 0; s < k; s++) {
      const T *sv = S.p[s];
      v0 -= es[s] * sv[i0];
      v1 -= es[s] * sv[i1];
    }
    // the first MQ columns of Q stay in registers for the dots below (read once)
    T qc0[MQ > 0 ? MQ : 1], qc1[MQ > 0 ? MQ : 1];
#pragma unroll
    for (int q = 0; q < MQ; q++)
      if (q < m) {
        qc0[q] = Q.p[q][i0];
        qc1[q] = Q.p[q][i1];
        v0 -= zq[q] * qc0[q];
        v1 -= zq[q] * qc1[q];
      }
    for (int q = MQ; q < m; q++) {
      const T *qv = Q.p[q];
      v0 -= zq[q] * qv[i0];
      v1 -= zq[q] * qv[i1];
    }
    if (with_beta) {
      v0 += beta * p[i0];
      v1 += beta * p[i1];
    }
    p[i0] = v0;
    if (two) p[i1] = v1;
#pragma unroll
    for (int d = 0; d < NA; d++) {
      if (d < m && d < nd) {
        if (d < MQ) {
          acc[d] += qc0[d < MQ ? d : 0] * v0;
          if (two) acc[d] += qc1[d < MQ ? d : 0] * v1;
        } else {
          acc[d] += Q.p[d][i0] * v0;
          if (two) acc[d] += Q.p[d][i1] * v1;
        }
      } else if (d < nd) {
        acc[d] += AQ.p[d - m][i0] * v0;
        if (two) acc[d] += AQ.p[d - m][i1] * v1;
      }
    }
  }
  if (MAXD > 0) bpart<T, NA>(acc, nd, part);
}

// ============================================================== PCG control kernels
__global__ void c_pcg_setup(DevCtl *c, double theta, int k, int m, int itmax, double tol_pcg, double tau, int exit_rule,
                            double xi, int eigtest) {
  if (threadIdx.x) return;
  c->theta = theta;
  c->k = k;
  c->m = m;
  c->itmax = itmax;
  c->tol_pcg = tol_pcg;
  c->tau = tau;
  c->exit_rule = exit_rule;
  c->xi = xi;
  c->eigtest = eigtest;
  c->its = 0;
  c->done = 0;
  c->reason = 0;
  c->first = 1;
}

__global__ void c_pcg_qr(DevCtl *c, const double *part, int nb, int m) {
  __shared__ double red[kMaxQ];
  reduce_parts(part, nb, m, red);
  if (threadIdx.x < m) c->Qr[threadIdx.x] = red[threadIdx.x];
}

// after k_pcg_init: g0, sigma, Q^T g, first-loop coefficients
__global__ void c_pcg_init(DevCtl *c, const double *part, int nb) {
  __shared__ double red[1 + kMaxK + kMaxQ];
  __shared__ GramLds G;
  const int k = c->k, m = c->m;
  reduce_parts(part, nb, 1 + k + m, red);
  stage_gram(c, k, G);
  if (threadIdx.x) return;
  c->gn = sqrt(red[0]);
  c->g0 = c->gn;
  for (int s = 0; s < k; s++) c->sig[s] = red[1 + s];
  for (int q = 0; q < m; q++) c->Qg[q] = red[1 + k + q];
  if (!(c->g0 > 0.0)) {  // zero right-hand side: s = 0 is the solution
    c->done = 1;
    c->reason = 1;
    return;
  }
  first_loop(c, k, red + 1, G);
}

// after the multi-dot (R^T c0 (k), Q^T c0 (m), g^T c0): second loop, CGS, rho, beta
__global__ void c_pcg_beta(DevCtl *c, const double *part, int nb) {
  if (c->done) return;
  __shared__ double red[kMaxK + kMaxQ + 1];
  __shared__ GramLds G;
  __shared__ double QS[kMaxQ * kMaxK], sig[kMaxK], Qg[kMaxQ], e[kMaxK];
  const int k = c->k, m = c->m;
  reduce_parts(part, nb, k + m + 1, red);
  for (int i = threadIdx.x; i < m * kMaxK; i += blockDim.x) QS[i] = c->QS[i];
  for (int i = threadIdx.x; i < k; i += blockDim.x) {
    sig[i] = c->sig[i];
    G.a[i] = c->a[i];
  }
  for (int i = threadIdx.x; i < m; i += blockDim.x) Qg[i] = c->Qg[i];
  stage_gram(c, k, G);
  if (threadIdx.x) return;
  for (int s = 0; s < k; s++) {
    double v = red[s];
    for (int t = 0; t < s; t++) v -= e[t] * G.M[t * kMaxK + s];
    const double b = v / G.alpha[s];
    c->b[s] = b;
    e[s] = G.a[s] + b;
    c->e[s] = e[s];
  }
  double rho1 = red[k + m];  // g^T c0
  for (int s = 0; s < k; s++) rho1 -= e[s] * sig[s];
  for (int q = 0; q < m; q++) {
    double z = red[k + q];
    for (int s = 0; s < k; s++) z -= e[s] * QS[q * kMaxK + s];
    c->zQ[q] = z;
    rho1 -= z * Qg[q];
  }
  if (c->first) {
    c->beta = 0.0;
    c->first = 0;
  } else {
    c->beta = rho1 / c->rho;
  }
  c->rho = rho1;
}

// after SpMV (p^T ap, p^T p) and k_pcg_newp (Q^T p, (AQ)^T p)  ->  zy = Q^T (A - theta I) p, p^T J p, gamma
__global__ void c_pcg_gamma(DevCtl *c, const double *part_s, int nbs, const double *part_p, int nbp) {
  if (c->done) return;
  __shared__ double red[2];
  __shared__ double rq[2 * kMaxQ];
  const int m = c->m;
  reduce_parts(part_s, nbs, 2, red, 0, false);  // waves 0 and 1, while the other two start on the m dots
  reduce_parts(part_p, nbp, 2 * m, rq, 2);
  if (threadIdx.x) return;
  const double th = c->theta;
  const double pap = red[0], pp = red[1];
  double pJp = pap - th * pp;
  for (int q = 0; q < m; q++) {
    const double qp = rq[q];
    c->zy[q] = rq[m + q] - th * qp;
    c->Qp[q] = qp;
    pJp -= qp * c->zy[q];
  }
  c->pJp = pJp;
  if (!(pJp > 0.0)) {
    c->done = 1;
    c->reason = 4;
    return;
  }
  c->gamma = c->rho / pJp;
}

// after k_pcg_update: ||g||, q, Q^T g, sigma
__global__ void c_pcg_q(DevCtl *c, const double *part, int nb) {
  if (c->done) return;
  __shared__ double red[3 + kMaxK + kMaxQ];
  const int k = c->k, m = c->m;
  reduce_parts(part, nb, 3 + k + m, red);
  if (threadIdx.x) return;
  c->gn = sqrt(red[0]);
  c->xAx = red[1];
  c->xx = red[2];
  c->q = (c->xx > 0.0) ? red[1] / red[2] : 0.0;
  for (int q = 0; q < m; q++) c->Qg[q] = red[3 + q];
  for (int s = 0; s < k; s++) c->sig[s] = red[3 + m + s];
}

// exit tests (Sec. 4.3) and, when continuing, first-loop coefficients
// Exit tests of the PCG iteration; posts the done flag of the iteration to the host (also when an earlier
// step of the iteration already ended the solve).
__global__ void c_pcg_exit(DevCtl *c, const double *part, int nb, int *hflag, int seq) {
  if (c->done) {
    if (threadIdx.x == 0) post_flag(hflag, 2 * seq + 1);
    return;
  }
  __shared__ double red[1];
  __shared__ GramLds G;
  __shared__ double sig[kMaxK];
  const int k = c->k;
  if (c->eigtest) reduce_parts(part, nb, 1, red);
  for (int i = threadIdx.x; i < k; i += blockDim.x) sig[i] = c->sig[i];
  stage_gram(c, k, G);
  if (threadIdx.x) return;
  c->its++;
  c->eigres = c->eigtest ? sqrt(red[0] / c->xx) : INFINITY;
  int why = -1;
  if (c->gn <= c->tol_pcg * c->g0) why = 1;
  else if (c->eigtest && c->eigres < c->tau * c->q) why = 2;
  else if (c->exit_rule == 1 && c->eigtest && c->gn <= c->xi * c->eigres) why = 3;
  else if (c->its >= c->itmax) why = 0;
  if (why >= 0) {
    c->done = 1;
    c->reason = why;
    post_flag(hflag, 2 * seq + 1);
    return;
  }
  post_flag(hflag, 2 * seq);
  first_loop(c, k, sig, G);
}

// ============================================================== generic combination
// out = cb0 * b0 + (cb1 ? *cb1 : 0) * b1 + sum_t lc[t] V_t  with cb0 = cb0c * (cb0d ? *cb0d : 1);
// lc = sgn * coef[t] (coef from device);  dots of out with W (nd) into part.
template <typename T, int MAXD>
__global__ __launch_bounds__(kBlock) void k_comb(int n, T *out, const T *b0, double cb0c, const double *cb0d, const T *b1,
                                                 const double *cb1, int nt, VList<T> V, const double *coef, double sgn,
                                                 int nd, VList<T> W, double *part, const int *gate) {
  if (gate && *gate) return;
  const T c0 = (T)(cb0c * (cb0d ? *cb0d : 1.0));
  const T c1 = cb1 ? (T)(*cb1) : T(0);
  // the coefficients, read once per workgroup (the stores to out could alias them)
  __shared__ T lc[kMaxVec];
  for (int t = threadIdx.x; t < nt; t += kBlock) lc[t] = (T)(sgn * coef[t]);
  __syncthreads();
  T acc[MAXD > 0 ? MAXD : 1];
#pragma unroll
  for (int d = 0; d < (MAXD > 0 ? MAXD : 1); d++) acc[d] = T(0);
  // two rows a grid stride apart per pass, so that the loads of both are in flight together; the rows
  // still enter each sum in grid-stride order.  W is read after out is stored (W may hold out).
  const int stride = gridDim.x * blockDim.x;
  for (int i0 = blockIdx.x * blockDim.x + threadIdx.x; i0 < n; i0 += 2 * stride) {
    const int i1 = i0 + stride < n ? i0 + stride : i0;
    const bool two = i0 + stride < n;
    T v0 = b0 ? c0 * b0[i0] : T(0), v1 = b0 ? c0 * b0[i1] : T(0);
    if (b1) {
      v0 += c1 * b1[i0];
      v1 += c1 * b1[i1];
    }
    for (int t = 0; t < nt; t++) {
      const T *vt = V.p[t];
      v0 += lc[t] * vt[i0];
      v1 += lc[t] * vt[i1];
    }
    out[i0] = v0;
    if (two) out[i1] = v1;
#pragma unroll
    for (int d = 0; d < MAXD; d++)
      if (d < nd) {
        acc[d] += v0 * W.p[d][i0];
        if (two) acc[d] += v1 * W.p[d][i1];
      }
  }
  if (MAXD > 0) bpart<T, (MAXD > 0 ? MAXD : 1)>(acc, nd, part);
}

// ============================================================== outer step (double)
// x = u + s;  dots: Qt_c^T x (nq), x^T x, s^T r, s^T s
template <typename T, int MAXD>
__global__ __launch_bounds__(kBlock) void k_outer_add(int n, const double *u, const T *s, const double *r, double *x,
                                                      int nq, VList<double> Qt, double *part) {
  double acc[MAXD];
#pragma unroll
  for (int d = 0; d < MAXD; d++) acc[d] = 0.0;
  GRIDLOOP(i, n) {
    const double si = (double)s[i];
    const double xi = u[i] + si;
    x[i] = xi;
    acc[0] += xi * xi;
    acc[1] += si * r[i];
    acc[2] += si * si;
#pragma unroll
    for (int d = 3; d < MAXD; d++)
      if (d < 3 + nq) acc[d] += Qt.p[d - 3][i] * xi;
  }
  bpart<double, MAXD>(acc, 3 + nq, part);
}

// r = Au - theta u; ||r||^2; mirrors of u, Au, r in T
template <typename T>
__global__ __launch_bounds__(kBlock) void k_outer_resid(int n, const DevCtl *c, const double *u, const double *Au,
                                                        double *r, T *uT, T *AuT, T *rT, double *part) {
  const double th = c->otheta;
  double acc[1] = {0.0};
  GRIDLOOP(i, n) {
    const double ri = Au[i] - th * u[i];
    r[i] = ri;
    acc[0] += ri * ri;
    if (uT) {
      uT[i] = (T)u[i];
      AuT[i] = (T)Au[i];
      rT[i] = (T)ri;
    }
  }
  bpart<double, 1>(acc, 1, part);
}

__global__ void c_reduce_to(double *dst, const double *part, int nb, int D) {
  __shared__ double red[kPartSlots];
  reduce_parts(part, nb, D, red);
  if (threadIdx.x < D) dst[threadIdx.x] = red[threadIdx.x];
}

// after k_outer_add: oz = Qt^T x, ||x||^2, alpha = s^T r_old, ||s||^2
__global__ void c_outer_add(DevCtl *c, const double *part, int nb, int nq) {
  __shared__ double red[3 + kMaxQ];
  reduce_parts(part, nb, 3 + nq, red);
  if (threadIdx.x) return;
  c->onrm2 = red[0];
  c->oalpha = red[1];
  c->osn2 = red[2];
  for (int q = 0; q < nq; q++) c->oz[q] = red[3 + q];
}

// CGS coefficients of the next pass (dots of the previous comb) and the last norm
__global__ void c_outer_cgs(DevCtl *c, const double *part, int nb, int nq, int with_norm) {
  __shared__ double red[kMaxQ + 1];
  reduce_parts(part, nb, nq + with_norm, red);
  if (threadIdx.x) return;
  for (int q = 0; q < nq; q++) c->oz[q] = red[q];
  if (with_norm) c->onrm2 = red[nq];
}

__global__ void c_set(double *dst, double v) {
  if (threadIdx.x == 0) *dst = v;
}

__global__ void c_inv_sqrt(DevCtl *c, const double *src, double *dst) {
  if (threadIdx.x) return;
  *dst = 1.0 / sqrt(*src);
}

__global__ void c_outer_theta(DevCtl *c, const double *part, int nb) {
  __shared__ double red[1];
  reduce_parts(part, nb, 1, red);
  if (threadIdx.x == 0) c->otheta = red[0];
}

__global__ void c_outer_rn(DevCtl *c, const double *part, int nb) {
  __shared__ double red[1];
  reduce_parts(part, nb, 1, red);
  if (threadIdx.x == 0) c->orn = sqrt(red[0]);
}

// Gram blocks of the BFGS pairs (double).  Dots in part, in order:
//   if inserted: s_new^T r_t (t < k), s_t^T r_new (t < k-1), Qt_c^T s_new (c < nqt);   then u^T s_t (t < k).
__global__ void c_gram(DevCtl *c, const double *part, int nb, int shift, int inserted, int k, int nqt) {
  __shared__ double red[kPartSlots];
  const int D = (inserted ? (k + (k - 1) + nqt) : 0) + k;
  reduce_parts(part, nb, D, red);
  if (threadIdx.x) return;
  if (shift) {  // drop the oldest pair (index 0)
    for (int s = 0; s + 1 < kMaxK; s++) {
      c->alpha[s] = c->alpha[s + 1];
      for (int t = 0; t + 1 < kMaxK; t++) c->M[s * kMaxK + t] = c->M[(s + 1) * kMaxK + t + 1];
      for (int q = 0; q < kMaxQ; q++) c->QS[q * kMaxK + s] = c->QS[q * kMaxK + s + 1];
    }
  }
  int o = 0;
  if (inserted) {
    const int kn = k - 1;
    for (int t = 0; t < k; t++) c->M[kn * kMaxK + t] = red[o + t];
    o += k;
    for (int t = 0; t < kn; t++) c->M[t * kMaxK + kn] = red[o + t];
    o += kn;
    c->alpha[kn] = c->M[kn * kMaxK + kn];
    for (int q = 0; q < nqt; q++) c->QS[q * kMaxK + kn] = red[o + q];
    o += nqt;
  }
  for (int t = 0; t < k; t++) c->QS[nqt * kMaxK + t] = red[o + t];
}

// out = r_k - r_{k+1} (the stored vector of the full BFGS pair, eq. (2.1) with y_k = r_{k+1} - r_k)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_ydiff(int n, const double *rk, const double *rk1, T *out) {
  GRIDLOOP(i, n) out[i] = (T)(rk[i] - rk1[i]);
}

__global__ void c_outer_y(DevCtl *c, const double *part, int nb) {
  __shared__ double red[2];
  reduce_parts(part, nb, 2, red);
  if (threadIdx.x) return;
  c->oya = red[0];
  c->oyn2 = red[1];
}

// ------------------------------------------------------------------ Jacobi-Davidson (Sec. 6)
// new column m of H = V^T A V from the dots v_i^T (A v_m), i <= m (mirrored into row m)
__global__ void c_jd_col(DevCtl *c, const double *part, int nb, int m) {
  __shared__ double red[kJdMax];
  reduce_parts(part, nb, m + 1, red);
  if (threadIdx.x) return;
  for (int i = 0; i <= m; i++) {
    c->jH[i * kJdMax + m] = red[i];
    c->jH[m * kJdMax + i] = red[i];
  }
}

// Rayleigh-Ritz on the m x m matrix H: Jacobi rotations, each zeroing one off-diagonal
// entry of a working copy, sweep after sweep until the off-diagonal mass is negligible;
// the rotations accumulate in E (eigenvectors as columns).  Ritz values go to jev in
// ascending order with their vectors in jY; theta = the smallest.  One thread: m <= 16.
__global__ void c_jd_rr(DevCtl *c, int m) {
  __shared__ double a[kJdMax][kJdMax], E[kJdMax][kJdMax];
  __shared__ int ord[kJdMax];
  if (threadIdx.x) return;
  for (int i = 0; i < m; i++)
    for (int q = 0; q < m; q++) {
      a[i][q] = c->jH[i * kJdMax + q];
      E[i][q] = i == q ? 1.0 : 0.0;
    }
  for (int sweep = 0; sweep < 64; sweep++) {
    double off = 0.0, all = 0.0;
    for (int i = 0; i < m; i++)
      for (int q = 0; q < m; q++) {
        const double x = a[i][q] * a[i][q];
        all += x;
        if (i != q) off += x;
      }
    if (!(off > 1e-30 * all)) break;
    for (int pp = 0; pp + 1 < m; pp++)
      for (int qq = pp + 1; qq < m; qq++) {
        const double apq = a[pp][qq];
        if (apq == 0.0) continue;
        const double w = (a[qq][qq] - a[pp][pp]) / (2.0 * apq);
        const double t = (w < 0.0 ? -1.0 : 1.0) / (fabs(w) + sqrt(w * w + 1.0));
        const double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
        for (int i = 0; i < m; i++) {  // columns pp, qq
          const double x = a[i][pp], y = a[i][qq];
          a[i][pp] = cs * x - sn * y;
          a[i][qq] = sn * x + cs * y;
        }
        for (int i = 0; i < m; i++) {  // rows pp, qq
          const double x = a[pp][i], y = a[qq][i];
          a[pp][i] = cs * x - sn * y;
          a[qq][i] = sn * x + cs * y;
        }
        for (int i = 0; i < m; i++) {
          const double x = E[i][pp], y = E[i][qq];
          E[i][pp] = cs * x - sn * y;
          E[i][qq] = sn * x + cs * y;
        }
      }
  }
  for (int i = 0; i < m; i++) ord[i] = i;
  for (int i = 0; i < m; i++) {  // selection of the ascending order
    int best = i;
    for (int q = i + 1; q < m; q++)
      if (a[ord[q]][ord[q]] < a[ord[best]][ord[best]]) best = q;
    const int tmp = ord[i];
    ord[i] = ord[best];
    ord[best] = tmp;
  }
  for (int cc = 0; cc < m; cc++) {
    c->jev[cc] = a[ord[cc]][ord[cc]];
    for (int i = 0; i < m; i++) c->jY[cc * kJdMax + i] = E[i][ord[cc]];
  }
  c->otheta = c->jev[0];
}

// after a thick restart with the mmin smallest Ritz vectors, H is their Ritz values
__global__ void c_jd_restart(DevCtl *c, int mmin) {
  if (threadIdx.x) return;
  for (int i = 0; i < kJdMax; i++)
    for (int q = 0; q < kJdMax; q++) c->jH[i * kJdMax + q] = (i == q && i < mmin) ? c->jev[i] : 0.0;
}

// Gram blocks from scratch, rows row0..row0+nrows-1 of M (kind 0, s_s^T r_t) or of Q^T S (kind 1)
__global__ void c_gram_rows(DevCtl *c, const double *part, int nb, int k, int kind, int row0, int nrows) {
  __shared__ double red[kPartSlots];
  reduce_parts(part, nb, nrows * k, red);
  if (threadIdx.x) return;
  for (int a = 0; a < nrows; a++)
    for (int t = 0; t < k; t++) {
      if (kind == 0) c->M[(row0 + a) * kMaxK + t] = red[a * k + t];
      else c->QS[(row0 + a) * kMaxK + t] = red[a * k + t];
    }
  if (kind == 0)
    for (int a = 0; a < nrows; a++) c->alpha[row0 + a] = c->M[(row0 + a) * kMaxK + row0 + a];
}

// first-loop coefficients from sigma = S^T g and Q^T g (standalone preconditioner apply)
__global__ void c_prec_a(DevCtl *c, const double *part, int nb, int k, int m) {
  __shared__ double red[kMaxK + kMaxQ];
  __shared__ GramLds G;
  reduce_parts(part, nb, k + m, red);
  stage_gram(c, k, G);
  if (threadIdx.x) return;
  c->k = k;
  c->m = m;
  c->done = 0;
  c->first = 1;
  for (int s = 0; s < k; s++) c->sig[s] = red[s];
  for (int q = 0; q < m; q++) c->Qg[q] = red[k + q];
  first_loop(c, k, red, G);
}

// ============================================================== DACG kernels (Sec. 4.1)
// x = x' * inv, Ax = Ax' * inv (when inv != 0), g = Ax - q x with q = xAx/xx of the scaled vector
// dots: x^T x, x^T Ax  (q is formed by the control kernel from the previous dots)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_dacg_scale(int n, const DevCtl *c, T *x, T *Ax, double *part) {
  if (c->ddone) return;
  const T inv = (T)c->dinv;
  T acc[2] = {T(0), T(0)};
  GRIDLOOP(i, n) {
    T xi = x[i], ai = Ax[i];
    if (inv != T(0)) {
      xi *= inv;
      ai *= inv;
      x[i] = xi;
      Ax[i] = ai;
    }
    acc[0] += xi * xi;
    acc[1] += xi * ai;
  }
  bpart<T, 2>(acc, 2, part);
}

// Convergence test ||g|| <= tol q ||x|| (or the iteration cap); posts the flag of the iteration to the host.
// Runs in the last block of the kernel that produced the dots g^T g, x^T x, x^T A x (k_dacg_grad,
// k_dacg_move).  With fresh set (the FP64 iteration), x^T x and x^T A x of the stored iterate come along for
// this iteration's line search; the FP32 iteration keeps those of its step kernel.
__device__ __forceinline__ void dacg_conv(DevCtl *c, double *part, int nb, int *hflag, int seq, int fresh) {
  __shared__ double red[3];
  const bool ok = reduce_parts_fused(part, nb, 3, red);
  if (threadIdx.x) return;
  if (!ok) {
    c->err = 1;
    c->ddone = 1;
    post_flag(hflag, 2 * seq + 1);
    return;
  }
  if (fresh) {
    c->dxx = red[1];
    c->dxAx = red[2];
  }
  c->dgn = sqrt(red[0] / c->dxx);
  if (c->dgn < 0.9 * c->dbest) {
    c->dbest = c->dgn;
    c->dbest_it = c->dits;
  }
  // stall (float only): no 10 % gain for dstall iterations while within 10x of the target, i.e.
  // at the float residual floor, which can sit above tol q when q is small against ||A||
  const bool stall = c->dstall > 0 && c->dits - c->dbest_it >= c->dstall && c->dbest <= 10.0 * c->dtol * c->dq;
  if (stall) c->dstalled = 1;
  if (c->dgn <= c->dtol * c->dq || c->dits >= c->ditmax || stall) c->ddone = 1;
  post_flag(hflag, 2 * seq + c->ddone);
}

// Scale the iterate (x = x' inv, Ax = Ax' inv when inv != 0: the norm of x' comes from the previous step),
// g = Ax - q x with the scale-invariant q = x'^T A x' / x'^T x'; dot g^T g.
// Dots g^T g, x^T x, x^T A x of the scaled iterate.
// The convergence test of the iteration (dacg_conv) runs in the last block; with the iteration done
// already, that block only posts the flag.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_dacg_grad(int n, DevCtl *c, T *x, T *Ax, T *g, double *part, int *hflag,
                                                      int seq, int fresh) {
  if (c->ddone) {
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) post_flag(hflag, 2 * seq + 1);
    return;
  }
  const T inv = (T)c->dinv;
  const T q = (T)c->dq;
  T acc[3] = {T(0), T(0), T(0)};
  GRIDLOOP(i, n) {
    T xi = x[i], ai = Ax[i];
    if (inv != T(0)) {
      xi *= inv;
      ai *= inv;
      x[i] = xi;
      Ax[i] = ai;
    }
    const T gi = ai - q * xi;
    g[i] = gi;
    acc[0] += gi * gi;
    acc[1] += xi * xi;
    acc[2] += xi * ai;
  }
  bpart<T, 3, true>(acc, 3, part);
  if (blockIdx.x == gridDim.x - 1) dacg_conv(c, part, gridDim.x, hflag, seq, fresh);
}

__global__ void c_dacg_q(DevCtl *c, const double *part, int nb) {
  if (c->ddone) return;
  __shared__ double red[2];
  reduce_parts(part, nb, 2, red);
  if (threadIdx.x) return;
  c->dxx = red[0];
  c->dxAx = red[1];
  c->dq = red[1] / red[0];
}

// after multi-dot (Qt^T c0 (nq), g^T c0): zQ, gamma, beta
// dots, in order: Qt^T g (nq), Qt^T c0 (nq), g^T c0
__global__ void c_dacg_beta(DevCtl *c, const double *part, int nb, int nq) {
  if (c->ddone) return;
  __shared__ double red[2 * kMaxQ + 1];
  reduce_parts(part, nb, 2 * nq + 1, red);
  if (threadIdx.x) return;
  // gamma = g^T h with h = c0 - Qt zQ and g orthogonal to Qt up to rounding: g^T h = g^T c0 - (Qt^T g)^T zQ
  double gam = red[2 * nq];
  for (int q = 0; q < nq; q++) {
    c->Qg[q] = red[q];
    c->zQ[q] = red[nq + q];
    gam -= red[nq + q] * red[q];
  }
  c->beta = (c->dits == 0 || c->dgamma_prev == 0.0) ? 0.0 : gam / c->dgamma_prev;
  c->dgamma = gam;
}

// after the d update (dots d^T Ax, d^T x, d^T d) and SpMV Ad = A d (dot d^T Ad)
__global__ void c_dacg_alpha(DevCtl *c, const double *part_s, int nbs, const double *part_d, int nbd, int fused) {
  if (c->ddone) return;
  __shared__ double red[1];
  __shared__ double rd[3];
  reduce_parts(part_s, nbs, 1, red, 0, false);  // wave 0, while waves 1-3 take d's three dots
  reduce_parts(part_d, nbd, 3, rd, 1);
  if (threadIdx.x) return;
  const double dAd = red[0], dAx = rd[0], xd = rd[1], dd = rd[2];
  const double xAx = c->dxAx, xx = c->dxx;
  const double bA = dAx;  // d^T A x
  // minimiser of q(x + a d): A2 a^2 + B2 a + C2 = 0 (closed form), the root with the smaller quotient
  const double A2 = dAd * xd - bA * dd, B2 = dAd * xx - xAx * dd, C2 = bA * xx - xAx * xd;
  double r1, r2;
  if (A2 == 0.0) {
    r1 = r2 = (B2 != 0.0) ? -C2 / B2 : 0.0;
  } else {
    double disc = B2 * B2 - 4.0 * A2 * C2;
    if (disc < 0.0) disc = 0.0;
    const double tq = -0.5 * (B2 + (B2 >= 0.0 ? 1.0 : -1.0) * sqrt(disc));
    r1 = tq / A2;
    r2 = (tq != 0.0) ? C2 / tq : r1;
  }
  const double q1 = (xAx + 2 * r1 * bA + r1 * r1 * dAd) / (xx + 2 * r1 * xd + r1 * r1 * dd);
  const double q2 = (xAx + 2 * r2 * bA + r2 * r2 * dAd) / (xx + 2 * r2 * xd + r2 * r2 * dd);
  const double a = (q2 < q1) ? r2 : r1;
  c->dalpha = a;
  if (!fused) return;
  // the next iterate x + a d: its squared norm and x^T A x from this step's dots, all taken on the stored
  // vectors (equal in exact arithmetic to the dots of the updated ones, nothing carried over from earlier
  // steps); k_dacg_move scales it to unit norm with them
  const double nxx = xx + 2 * a * xd + a * a * dd, nxAx = xAx + 2 * a * bA + a * a * dAd;
  const double inv = 1.0 / sqrt(nxx);
  c->dinv = inv;
  c->dq = nxAx / nxx;
  c->dxx = nxx * inv * inv;
  c->dxAx = nxAx * inv * inv;
  c->dgamma_prev = c->dgamma;
  c->dits++;
}

// x' = (x + a d) inv, Ax' = (Ax + a Ad) inv (inv and q from c_dacg_alpha), g = Ax' - q x'; dots g^T g,
// x'^T x', x'^T A x'.  FP64 only: in FP32 the quotient of the unrounded step differs from that of the stored
// vectors by about the float epsilon times ||A||, which would put a floor under ||g||
__global__ __launch_bounds__(kBlock) void k_dacg_move(int n, DevCtl *c, double *x, double *Ax, const double *d,
                                                      const double *Ad, double *g, double *part, int *hflag, int seq) {
  if (c->ddone) {
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) post_flag(hflag, 2 * seq + 1);
    return;
  }
  const double a = c->dalpha, inv = c->dinv, q = c->dq;
  double acc[3] = {0.0, 0.0, 0.0};
  // two rows a grid stride apart per pass (loads of both in flight together; fp64 13.7 -> 13.1 us, no gain
  // in the fp32 step kernels); the sums still take the rows in grid-stride order
  const int stride = gridDim.x * blockDim.x;
  for (int i0 = blockIdx.x * blockDim.x + threadIdx.x; i0 < n; i0 += 2 * stride) {
    const bool two = i0 + stride < n;
    const int ii[2] = {i0, two ? i0 + stride : i0};
    double xv[2], av[2], dv[2], adv[2];
#pragma unroll
    for (int u = 0; u < 2; u++) {
      xv[u] = x[ii[u]];
      av[u] = Ax[ii[u]];
      dv[u] = d[ii[u]];
      adv[u] = Ad[ii[u]];
    }
#pragma unroll
    for (int u = 0; u < 2; u++) {
      if (u == 1 && !two) break;
      const int i = ii[u];
      const double xi = (xv[u] + a * dv[u]) * inv;
      const double ai = (av[u] + a * adv[u]) * inv;
      x[i] = xi;
      Ax[i] = ai;
      const double gi = ai - q * xi;
      g[i] = gi;
      acc[0] += gi * gi;
      acc[1] += xi * xi;
      acc[2] += xi * ai;
    }
  }
  bpart<double, 3, true>(acc, 3, part);
  if (blockIdx.x == gridDim.x - 1) dacg_conv(c, part, gridDim.x, hflag, seq, 1);
}

// next step, in the last block of k_dacg_step: inv = 1/||x'||, q, and the dots of the scaled iterate
__device__ __forceinline__ void dacg_next(DevCtl *c, double *part, int nb) {
  __shared__ double red[2];
  const bool ok = reduce_parts_fused(part, nb, 2, red);
  if (threadIdx.x) return;
  if (!ok) {
    c->err = 1;
    c->ddone = 1;
    return;
  }
  const double inv = 1.0 / sqrt(red[0]);
  c->dinv = inv;
  c->dq = red[1] / red[0];
  c->dxx = red[0] * inv * inv;
  c->dxAx = red[1] * inv * inv;
  c->dgamma_prev = c->dgamma;
  c->dits++;
}

// x' = x + a d, Ax' = Ax + a Ad; dots x'^T x', x'^T A x' (reduced by dacg_next in the last block)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_dacg_step(int n, DevCtl *c, T *x, T *Ax, const T *d, const T *Ad,
                                                      double *part) {
  if (c->ddone) return;
  const T a = (T)c->dalpha;
  T acc[2] = {T(0), T(0)};
  GRIDLOOP(i, n) {
    const T xi = x[i] + a * d[i];
    const T ai = Ax[i] + a * Ad[i];
    x[i] = xi;
    Ax[i] = ai;
    acc[0] += xi * xi;
    acc[1] += xi * ai;
  }
  bpart<T, 2, true>(acc, 2, part);
  if (blockIdx.x == gridDim.x - 1) dacg_next(c, part, gridDim.x);
}

__global__ void c_dacg_setup(DevCtl *c, double tol, int itmax, int stall) {
  if (threadIdx.x) return;
  c->dtol = tol;
  c->ditmax = itmax;
  c->dbest = 1e300;
  c->dbest_it = 0;
  c->dstall = stall;
  c->dstalled = 0;
  c->dits = 0;
  c->ddone = 0;
  c->dinv = 0.0;
  c->dgamma_prev = 0.0;
}

// ============================================================== IC(0) factor (device, level by level)
__global__ void k_ic0_gather(int nnzL, const int *map, const double *val, double *Lv) {
  GRIDLOOP(q, nnzL) Lv[q] = val[map[q]];
}

// rows of one level: L_ij = (A_ij - sum_{m<j} L_im L_jm)/L_jj ; L_ii = sqrt((1+a) A_ii - sum L_im^2)
__global__ void k_ic0_level(int r0, int r1, const int *rows, const int *Lrp, const int *Lci, double *Lv, double shift,
                            int *fail) {
  const int pos = r0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (pos >= r1) return;
  const int i = rows[pos];
  const int e0 = Lrp[i], ed = Lrp[i + 1] - 1;
  double dsum = 0.0;
  for (int e = e0; e < ed; e++) {
    const int j = Lci[e];
    double s = Lv[e];
    int p = e0, q = Lrp[j];
    const int qend = Lrp[j + 1] - 1;
    while (p < e && q < qend) {
      const int cp = Lci[p], cq = Lci[q];
      if (cp == cq) {
        s -= Lv[p] * Lv[q];
        p++;
        q++;
      } else if (cp < cq) {
        p++;
      } else {
        q++;
      }
    }
    s /= Lv[qend];
    Lv[e] = s;
    dsum += s * s;
  }
  const double d = Lv[ed] * (1.0 + shift) - dsum;
  if (!(d > 0.0)) {
    atomicOr(fail, 1);
    Lv[ed] = 1.0;
  } else {
    Lv[ed] = sqrt(d);
  }
}

__global__ void k_gather_d(int n, const int *map, const double *src, double *dst) {
  GRIDLOOP(q, n) dst[q] = src[map[q]];
}

// values of a block schedule: dst[q] = src[map[q]] (0 where map < 0), in precision T
template <typename T>
__global__ void k_gather_blk(int m, const int *map, const double *src, T *dst) {
  GRIDLOOP(q, m) {
    const int j = map[q];
    dst[q] = j >= 0 ? (T)src[j] : (j == -2 ? T(-1) : T(0));  // -2: a virtual row's partial sum
  }
}

// values of a level-compressed system from the factor values v of its direction (SolveSys)
__global__ void k_sys_values(int nnz, const int *direct, const int *tp, const int *ta, const int *tb, const int *tc,
                             const double *v, double *out) {
  GRIDLOOP(e, nnz) {
    double x = direct[e] >= 0 ? v[direct[e]] : 0.0;
    for (int t = tp[e]; t < tp[e + 1]; t++) x -= v[ta[t]] * v[tb[t]] / v[tc[t]];
    out[e] = x;
  }
}
__global__ void k_sys_m(int nm, const int *ma, const int *mc, const double *v, double *out) {
  GRIDLOOP(t, nm) out[t] = v[ma[t]] / v[mc[t]];
}

// reciprocal diagonal of a block schedule: dst[k] = 1 / src[map[k]] (rounded once, in double)
template <typename T>
__global__ void k_gather_rdiag(int m, const int *map, const double *src, T *dst) {
  GRIDLOOP(q, m) dst[q] = map[q] >= 0 ? (T)(1.0 / src[map[q]]) : T(1);  // -1: a virtual row
}

// ============================================================== output helpers
__global__ void k_absmax(int n, const double *v, double *part) {
  double m = 0.0;
  GRIDLOOP(i, n) m = fmax(m, fabs(v[i]));
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// sign of the first entry with |v_i| > 1e-12 max|v| (per block: smallest such index, encoded with its sign)
__global__ void k_firstbig(int n, const double *v, const double *part_max, int nbm, double *part) {
  __shared__ double vmax_s;
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int b = 0; b < nbm; b++) m = fmax(m, part_max[b]);
    vmax_s = m;
  }
  __syncthreads();
  const double thr = 1e-12 * vmax_s;
  long long best = (long long)n;
  GRIDLOOP(i, n) if (fabs(v[i]) > thr && i < best) best = i;
  for (int off = 32; off > 0; off >>= 1) {
    long long o = __shfl_xor(best, off, 64);
    best = o < best ? o : best;
  }
  __shared__ long long red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long b = red[0];
    for (int w = 1; w < 4; w++) b = red[w] < b ? red[w] : b;
    part[blockIdx.x] = (double)b;
  }
}

__global__ void k_sign_copy(int n, const double *v, const double *part_idx, int nb, double *out) {
  __shared__ double sg;
  if (threadIdx.x == 0) {
    double b = (double)n;
    for (int k = 0; k < nb; k++) b = fmin(b, part_idx[k]);
    const long long i = (long long)b;
    sg = (i < n && v[i] < 0.0) ? -1.0 : 1.0;
  }
  __syncthreads();
  GRIDLOOP(i, n) out[i] = sg * v[i];
}

// ============================================================== backward kernels
// g_vals[e=(a,b)] += sum_i ge_i v_i[a] v_i[b]
__global__ void k_grad_lambda(int n, const int *rp, const int *ci, int p, const double *V, const double *ge,
                              double *gv) {
  GRIDLOOP(a, n) {
    for (int e = rp[a]; e < rp[a + 1]; e++) {
      const int b = ci[e];
      double s = 0.0;
      for (int i = 0; i < p; i++) s += ge[i] * V[(size_t)i * n + a] * V[(size_t)i * n + b];
      gv[e] += s;
    }
  }
}

// g_vals[e=(a,b)] -= 1/2 (xi[a] v[b] + v[a] xi[b])
__global__ void k_grad_vec(int n, const int *rp, const int *ci, const double *v, const double *xi, double *gv) {
  GRIDLOOP(a, n) {
    const double xa = xi[a], va = v[a];
    for (int e = rp[a]; e < rp[a + 1]; e++) {
      const int b = ci[e];
      gv[e] -= 0.5 * (xa * v[b] + va * xi[b]);
    }
  }
}

// coefficients (v_j^T G)/(lambda_j - lambda_i) for j < i, from the dots in part
__global__ void c_adj_coef(DevCtl *c, const double *part, int nb, int ni, const double *lam, int i) {
  __shared__ double red[kMaxQ];
  reduce_parts(part, nb, ni, red);
  if (threadIdx.x < ni) c->bz[threadIdx.x] = red[threadIdx.x] / (lam[threadIdx.x] - lam[i]);
}

}  // namespace

// ================================================================== context
struct bnx_ctx {
  int n = 0, nnz = 0, device_ptrs = 0;
  hipStream_t st = nullptr;
  std::string err;
  Analysis an;                 // A, and the IC(0) pattern tril(A)
  Analysis anT;                // pattern of the last IC(lfil, tau_IC) factor
  const Analysis *ta = nullptr;  // pattern the device triangular structures hold (&an or &anT)
  int group = 8;
  // device arrays
  int *rp = nullptr, *ci = nullptr;
  double *val = nullptr;
  float *val32 = nullptr;
  // SELL-64 copy of A (when its padding is modest)
  int *ell_ptr = nullptr, *ell_len = nullptr, *ell_col = nullptr, *ell_map = nullptr;
  double *ell_v64 = nullptr;
  float *ell_v32 = nullptr;
  int ell_size = 0;
  int *Lrp = nullptr, *Lci = nullptr, *mapL = nullptr, *Ltrp = nullptr, *Ltci = nullptr, *mapLt = nullptr;
  int *levL = nullptr, *levLt = nullptr;
  double *Lv = nullptr, *Ltv = nullptr;
  float *Lv32 = nullptr, *Ltv32 = nullptr;
  // block schedules of the LDS-staged solve: [0] forward (L), [1] backward (L^T); per precision
  struct BlkDev {
    int n = 0, npad = 0, nblocks = 0, ell = 0, nexp = 0, nr = kNR;
    int *bptr = nullptr, *brows = nullptr, *iptr = nullptr, *isrc = nullptr;
    int *eptr = nullptr, *erank = nullptr, *orow = nullptr, *oslot = nullptr;
    int *perm = nullptr, *slice_ptr = nullptr, *slice_nnz = nullptr, *ref = nullptr;
    int *valmap = nullptr, *diagmap = nullptr, *cnt = nullptr, *ref4 = nullptr, *valmap4 = nullptr;
    int *mjr = nullptr, *mtr = nullptr, mw = 0;  // rank-order right-hand-side transform (compressed systems)
    double *diag64 = nullptr, *val64 = nullptr, *val4_64 = nullptr;
    float *diag32 = nullptr, *val32 = nullptr, *val4_32 = nullptr;
  } blk[2][2];  // [direction][0 = fp64 LDS capacity, 1 = fp32 LDS capacity]
  // Level-compressed solve systems ([0] forward, [1] backward; compress_system), used by the
  // FP32 solves when lps is set (in FP64 the compressed kernel gains nothing measurable); the
  // other solves use the factor's own rows (Lrp/Lci/Lv and Ltrp/Ltci/Ltv).
  bool lps = false;
  Analysis anS;  // their patterns and levels: forward system in L*, backward system in Lt*
  struct SysDev {
    int nnz = 0, nm = 0;
    int *rp = nullptr, *ci = nullptr, *lev = nullptr;
    int *direct = nullptr, *tp = nullptr, *ta = nullptr, *tb = nullptr, *tc = nullptr;
    int *mp = nullptr, *mj = nullptr, *ma = nullptr, *mc = nullptr;
    double *v = nullptr, *mv = nullptr;
    float *v32 = nullptr, *mv32 = nullptr;
  } sys[2];
  // export buffers of the block solves, per precision two halves of the largest nexp of its two
  // schedules, and their ticket counters ([0..1] fp64, [2..3] fp32); a launch uses one half and resets
  // the other for the next launch of the same precision (blk_seq counts them)
  double *blk_exp64 = nullptr;
  float *blk_exp32 = nullptr;
  int blk_nexp64 = 0, blk_nexp32 = 0;
  int *blk_cnt = nullptr;
  mutable long long blk_seq[2] = {0, 0};
  int *probe_flags = nullptr;  // latency probe flags (allocated on first use)
  void *scratch = nullptr;     // device address of this device's copy of the no-allocation scratch array
  DevCtl *ctl = nullptr;
  DevCtl *hctl = nullptr;  // pinned readback
  double *part = nullptr;
  int *counter = nullptr;
  int *dflag = nullptr;    // device int scratch
  int *hflag = nullptr;    // pinned, mapped
  int *dhflag = nullptr;   // device address of hflag
  bool factored = false, solved = false;
  double shift_used = 0.0, t_factor = 0.0;
  int trsv_mode = 0, sf_waves = 0;  // 0: window from the level sizes
  double adj_tol = 1e-12;
  int adj_itmax = 2000;
  // last solve
  int p_last = 0;
  std::vector<double> evals_last;
  double *evecs_last = nullptr;  // n x p fp64 (sorted, signed)
  int prec_last = 0;
  std::vector<void *> owned;
  Profiler prof;

  template <typename T>
  T *alloc(size_t count) {
    void *q = nullptr;
    if (count == 0) count = 1;
    if (hipMalloc(&q, count * sizeof(T)) != hipSuccess) throw ApiError{BNX_E_NOMEM, "device allocation failed"};
    owned.push_back(q);
    return static_cast<T *>(q);
  }
  void release(void *q) {
    if (!q) return;
    auto it = std::find(owned.begin(), owned.end(), q);
    if (it != owned.end()) owned.erase(it);
    (void)hipFree(q);
  }
  ~bnx_ctx() {
    (void)hipStreamSynchronize(st);
    for (void *q : owned) (void)hipFree(q);
    if (hctl) (void)hipHostFree(hctl);
    if (hflag) (void)hipHostFree(hflag);
  }

  Launch launch() const {
    Launch L;
    L.prof = const_cast<Profiler *>(&prof);
    L.st = st;
    L.nb = kNBMax;
    L.ctl = ctl;
    L.part = part;
    L.counter = counter;
    L.trsv_mode = trsv_mode;
    L.sf_waves = sf_waves;
    return L;
  }
  template <typename T>
  Mat<T> mat() const;
  template <typename T>
  Tri<T> tri(bool lower) const;
  void sync() {
    HIPCHK(hipStreamSynchronize(st));
    if (prof.on) prof.drain();
  }
  DevCtl readctl() {
    HIPCHK(hipMemcpyAsync(hctl, ctl, sizeof(DevCtl), hipMemcpyDeviceToHost, st));
    sync();
    return *hctl;
  }
};

template <>
Mat<double> bnx_ctx::mat<double>() const {
  Mat<double> M;
  M.n = n;
  M.rp = rp;
  M.ci = ci;
  M.v = val;
  M.group = group;
  if (ell_ptr) {
    M.ell_ptr = ell_ptr;
    M.ell_len = ell_len;
    M.ell_col = ell_col;
    M.ell_val = ell_v64;
  }
  return M;
}
template <>
Mat<float> bnx_ctx::mat<float>() const {
  Mat<float> M;
  M.n = n;
  M.rp = rp;
  M.ci = ci;
  M.v = val32;
  M.group = group;
  if (ell_ptr) {
    M.ell_ptr = ell_ptr;
    M.ell_len = ell_len;
    M.ell_col = ell_col;
    M.ell_val = ell_v32;
  }
  return M;
}
template <>
Tri<double> bnx_ctx::tri<double>(bool lower) const {
  Tri<double> F;
  {
    const BlkDev &b = blk[lower ? 0 : 1][0];
    F.blk.n = b.n;
    F.blk.nr = b.nr;
    F.blk.npad = b.npad;
    F.blk.nblocks = b.nblocks;
    F.blk.nexp = b.nexp;
    F.blk.ell = b.ell;
    F.blk.bptr = b.bptr;
    F.blk.brows = b.brows;
    F.blk.iptr = b.iptr;
    F.blk.isrc = b.isrc;
    F.blk.eptr = b.eptr;
    F.blk.erank = b.erank;
    F.blk.orow = b.orow;
    F.blk.oslot = b.oslot;
    F.blk.perm = b.perm;
    F.blk.slice_ptr = b.slice_ptr;
    F.blk.slice_nnz = b.slice_nnz;
    F.blk.ref = b.ref;
    F.blk.diag = b.diag64;
    F.blk.val = b.val64;
    F.blk.cnt = b.cnt;
    F.blk.ref4 = b.ref4;
    F.blk.val4 = b.val4_64;
  }
  F.blk_exp = blk_exp64;
  F.blk_nexp = blk_nexp64;
  F.blk_cnt = blk_cnt;
  F.blk_seq = &blk_seq[0];
  F.n = n;
  F.lower = lower;
  F.rp = lower ? Lrp : Ltrp;
  F.ci = lower ? Lci : Ltci;
  F.v = lower ? Lv : Ltv;
  F.lev_rows = lower ? levL : levLt;
  const Analysis &la = *ta;
  const Levels &lv = lower ? la.levL : la.levLt;
  F.lev_ptr = &lv.ptr;
  F.nlev = lv.nlev;
  F.max_rows = lv.max_rows;
  return F;
}
template <>
Tri<float> bnx_ctx::tri<float>(bool lower) const {
  Tri<float> F;
  {
    const BlkDev &b = blk[lower ? 0 : 1][1];
    F.blk.n = b.n;
    F.blk.nr = b.nr;
    F.blk.npad = b.npad;
    F.blk.nblocks = b.nblocks;
    F.blk.nexp = b.nexp;
    F.blk.ell = b.ell;
    F.blk.bptr = b.bptr;
    F.blk.brows = b.brows;
    F.blk.iptr = b.iptr;
    F.blk.isrc = b.isrc;
    F.blk.eptr = b.eptr;
    F.blk.erank = b.erank;
    F.blk.orow = b.orow;
    F.blk.oslot = b.oslot;
    F.blk.perm = b.perm;
    F.blk.slice_ptr = b.slice_ptr;
    F.blk.slice_nnz = b.slice_nnz;
    F.blk.ref = b.ref;
    F.blk.diag = b.diag32;
    F.blk.val = b.val32;
    F.blk.cnt = b.cnt;
    F.blk.ref4 = b.ref4;
    F.blk.val4 = b.val4_32;
    F.blk.mjr = b.mjr;
    F.blk.mtr = b.mtr;
    F.blk.mw = b.mw;
  }
  F.blk_exp = blk_exp32;
  F.blk_nexp = blk_nexp32;
  F.blk_cnt = blk_cnt ? blk_cnt + 2 : nullptr;
  F.blk_seq = &blk_seq[1];
  F.n = n;
  F.lower = lower;
  if (lps) {
    const SysDev &S = sys[lower ? 0 : 1];
    F.rp = S.rp;
    F.ci = S.ci;
    F.v = S.v32;
    F.lev_rows = S.lev;
    F.M.mp = S.mp;
    F.M.mj = S.mj;
    F.M.mv = S.mv32;
  } else {
    F.rp = lower ? Lrp : Ltrp;
    F.ci = lower ? Lci : Ltci;
    F.v = lower ? Lv32 : Ltv32;
    F.lev_rows = lower ? levL : levLt;
  }
  const Analysis &la = lps ? anS : *ta;
  const Levels &lv = lower ? la.levL : la.levLt;
  F.lev_ptr = &lv.ptr;
  F.nlev = lv.nlev;
  F.max_rows = lv.max_rows;
  return F;
}

namespace {

int gridn(int n) { return grid_for((size_t)n, kNBMax); }

template <typename T>
VList<T> vl(std::initializer_list<const T *> ps) {
  VList<T> v{};
  int i = 0;
  for (const T *q : ps) v.p[i++] = q;
  return v;
}

// ------------------------------------------------------------------ generic comb launcher
template <typename T>
int comb(bnx_ctx *C, T *out, const T *b0, double cb0c, const double *cb0d, const T *b1, const double *cb1, int nt,
         const VList<T> &V, const double *coef, double sgn, int nd, const VList<T> &W, double *part,
         const int *gate) {
  const int nb = gridn(C->n);
  if (nd == 0)
    hipLaunchKernelGGL((k_comb<T, 0>), dim3(nb), dim3(kBlock), 0, C->st, C->n, out, b0, cb0c, cb0d, b1, cb1, nt, V,
                       coef, sgn, 0, W, part, gate);
  else if (nd <= 4)
    hipLaunchKernelGGL((k_comb<T, 4>), dim3(nb), dim3(kBlock), 0, C->st, C->n, out, b0, cb0c, cb0d, b1, cb1, nt, V,
                       coef, sgn, nd, W, part, gate);
  else
    hipLaunchKernelGGL((k_comb<T, kMaxQ + 1>), dim3(nb), dim3(kBlock), 0, C->st, C->n, out, b0, cb0c, cb0d, b1, cb1,
                       nt, V, coef, sgn, nd, W, part, gate);
  return nb;
}

// ------------------------------------------------------------------ workspace
template <typename T>
struct Work {
  int n = 0, kmax = 0, pcap = 0;
  T *p, *ap, *s, *g, *t, *c0, *z, *u, *Au, *r, *x, *Ax, *d, *Ad, *dg;
  T *S[kMaxK], *R[kMaxK];
  T *Qm;   // n x pcap mirror of converged vectors
  T *AQm;  // n x pcap: A times each of them
};

template <typename T>
void make_work(bnx_ctx *C, Work<T> &w, int kmax, int pcap) {
  const size_t n = C->n;
  w.n = C->n;
  w.kmax = kmax;
  w.pcap = pcap;
  T **vecs[] = {&w.p, &w.ap, &w.s, &w.g, &w.t, &w.c0, &w.z, &w.u, &w.Au, &w.r, &w.x, &w.Ax, &w.d, &w.Ad, &w.dg};
  for (T **v : vecs) *v = C->alloc<T>(n);
  for (int s = 0; s < kMaxK; s++) w.S[s] = w.R[s] = nullptr;
  for (int s = 0; s < kmax; s++) {
    w.S[s] = C->alloc<T>(n);
    w.R[s] = C->alloc<T>(n);
  }
  w.Qm = C->alloc<T>(n * (size_t)std::max(pcap, 1));
  w.AQm = C->alloc<T>(n * (size_t)std::max(pcap, 1));
}

template <typename T>
void free_work(bnx_ctx *C, Work<T> &w) {
  T *vecs[] = {w.p, w.ap, w.s, w.g, w.t, w.c0, w.z, w.u, w.Au, w.r, w.x, w.Ax, w.d, w.Ad, w.dg, w.Qm, w.AQm};
  for (T *v : vecs) C->release(v);
  for (int s = 0; s < w.kmax; s++) {
    C->release(w.S[s]);
    C->release(w.R[s]);
  }
}

// ------------------------------------------------------------------ lagged done-flag polling
// The host queues an iteration before it reads the flag of an earlier one, so the device never waits for it.
struct Poll {
  // Iteration flags: the device posts 2 seq + done into pinned host memory (seq numbers the iterations
  // from 1; done sticks once set), and the host, after queueing iteration seq, waits for the flag of
  // iteration seq - 1 by reading that memory.  No event sits in the stream between the kernels.
  bnx_ctx *C;
  int seq = 0;
  explicit Poll(bnx_ctx *c) : C(c) { __atomic_store_n(&C->hflag[0], 0, __ATOMIC_RELEASE); }
  int *flag() const { return C->dhflag; }
  int next() { return ++seq; }  // number of the iteration being queued
  // done flag as of iteration s (the device has run at least that far); should the stream drain with
  // the flag missing, the queued work failed
  int read(int s) {
    for (long spins = 1;; spins++) {
      const int v = __atomic_load_n(&C->hflag[0], __ATOMIC_ACQUIRE);
      if ((v >> 1) >= s) return v & 1;
      if ((spins & 1023) == 0) {
        const hipError_t q = hipStreamQuery(C->st);
        if (q == hipErrorNotReady) continue;
        const int w = __atomic_load_n(&C->hflag[0], __ATOMIC_ACQUIRE);
        if ((w >> 1) >= s) return w & 1;
        HIPCHK(q);  // a failed launch or a device fault
        throw ApiError{BNX_E_STATE, "iteration flag not posted by the device"};
      }
    }
  }
};

// ------------------------------------------------------------------ PCG on the correction equation
struct PcgParams {
  double theta = 0, tol_pcg = 1e-2, tau = 1e-8, xi = 0.1, sgn = -1.0;
  int itmax = 20, exit_rule = 1, eigtest = 1;
};

// Solves J s = sgn (I - QQ^T) r with J = (I-QQ^T)(A - theta I)(I-QQ^T); Q = m vectors; pairs S,R (k,
// chronological; Gram blocks already in ctl).  u, Au: for the eigen-residual test (eigtest).
template <typename T>
void pcg(bnx_ctx *C, Work<T> &w, const PcgParams &P, const T *r, int m, const VList<T> &Q, const VList<T> &AQ, int k,
         const VList<T> &S, const VList<T> &R, const T *u, const T *Au, T *s_out, int *its, int *reason) {
  const Launch L = C->launch();
  const int n = C->n;
  const int *gate = &C->ctl->done;
  DevCtl *c = C->ctl;
  Mat<T> A = C->mat<T>();
  Tri<T> Lf = C->tri<T>(true), Lt = C->tri<T>(false);
  hipLaunchKernelGGL(c_pcg_setup, dim3(1), dim3(64), 0, C->st, c, P.theta, k, m, P.itmax, P.tol_pcg, P.tau,
                     P.exit_rule, P.xi, P.eigtest);
  // Q^T r
  if (m > 0) {
    VList<T> rr{};
    for (int q = 0; q < m; q++) rr.p[q] = r;
    const int nb = launch_multidot<T, T>(L, n, m, Q, rr, area(L, 3), nullptr);
    hipLaunchKernelGGL(c_pcg_qr, dim3(1), dim3(kBlock), 0, C->st, c, area(L, 3), nb, m);
  }
  const int nbi = gridn(n);
  const int Di = 1 + k + m;
  T *t = P.eigtest ? w.t : nullptr;
  // accumulator count tiers: the widest one costs registers (and occupancy) a typical solve never uses
  if (Di <= 8)
    hipLaunchKernelGGL((k_pcg_init<T, 8>), dim3(nbi), dim3(kBlock), 0, C->st, n, c, P.sgn, r, m, Q, k, S, w.g, s_out,
                       t, area(L, 1));
  else if (Di <= 24)
    hipLaunchKernelGGL((k_pcg_init<T, 24>), dim3(nbi), dim3(kBlock), 0, C->st, n, c, P.sgn, r, m, Q, k, S, w.g,
                       s_out, t, area(L, 1));
  else
    hipLaunchKernelGGL((k_pcg_init<T, 1 + kMaxK + kMaxQ>), dim3(nbi), dim3(kBlock), 0, C->st, n, c, P.sgn, r, m, Q,
                       k, S, w.g, s_out, t, area(L, 1));
  hipLaunchKernelGGL(c_pcg_init, dim3(1), dim3(kBlock), 0, C->st, c, area(L, 1), nbi);

  VList<T> ly{}, lx{};
  ly.p[0] = w.p;
  lx.p[0] = w.p;
  VList<T> mdX{};  // c0 against R (k), Q (m), g
  for (int s = 0; s < k; s++) mdX.p[s] = R.p[s];
  for (int q = 0; q < m; q++) mdX.p[k + q] = Q.p[q];
  mdX.p[k + m] = w.g;
  const int Du = 3 + k + m;

  Poll poll(C);
  int l;
  for (l = 0; l <= P.itmax; l++) {
    // c0 = P0^ (g - R a)   (first loop fused into the forward solve)
    launch_trsv<T>(L, Lf, w.g, w.z, k, R, c->a, gate);
    launch_trsv<T>(L, Lt, w.z, w.c0, 0, R, nullptr, gate);
    int nbd = launch_mdot_list<T, T>(L, n, 1, w.c0, nullptr, k + m + 1, mdX, 0, area(L, 3), gate);
    hipLaunchKernelGGL(c_pcg_beta, dim3(1), dim3(kBlock), 0, C->st, c, area(L, 3), nbd);
    if (2 * m <= 8)
      hipLaunchKernelGGL((k_pcg_newp<T, 8>), dim3(nbi), dim3(kBlock), 0, C->st, n, c, w.c0, k, S, m, Q, w.p,
                         l > 0 ? 1 : 0, 2 * m, AQ, area(L, 8));
    else if (2 * m <= 24)
      hipLaunchKernelGGL((k_pcg_newp<T, 24>), dim3(nbi), dim3(kBlock), 0, C->st, n, c, w.c0, k, S, m, Q, w.p,
                         l > 0 ? 1 : 0, 2 * m, AQ, area(L, 8));
    else
      hipLaunchKernelGGL((k_pcg_newp<T, 2 * kMaxQ>), dim3(nbi), dim3(kBlock), 0, C->st, n, c, w.c0, k, S, m, Q, w.p,
                         l > 0 ? 1 : 0, 2 * m, AQ, area(L, 8));
    // y = J p
    int nbs = launch_spmv<T>(L, A, w.p, w.ap, 1, ly, 1, lx, area(L, 0), gate);
    hipLaunchKernelGGL(c_pcg_gamma, dim3(1), dim3(kBlock), 0, C->st, c, area(L, 0), nbs, area(L, 8), nbi);
    if (Du <= 8)
      hipLaunchKernelGGL((k_pcg_update<T, 8, 2, 5>), dim3(nbi), dim3(kBlock), 0, C->st, n, c, w.ap, w.p, m, Q, k, S, u,
                         Au, s_out, w.g, t, area(L, 1));
    else if (Du <= 24)
      // fp64: one row per pass with eight Q columns in registers; fp32: two rows with six (both fit the
      // four waves per SIMD the grid needs)
      hipLaunchKernelGGL((k_pcg_update<T, 24, sizeof(T) == 8 ? 1 : 2, sizeof(T) == 8 ? 8 : 6>), dim3(nbi),
                         dim3(kBlock), 0, C->st, n, c, w.ap, w.p, m, Q, k, S, u, Au, s_out, w.g, t, area(L, 1));
    else
      hipLaunchKernelGGL((k_pcg_update<T, 3 + kMaxK + kMaxQ, 1, 0>), dim3(nbi), dim3(kBlock), 0, C->st, n, c, w.ap,
                         w.p, m, Q, k, S, u, Au, s_out, w.g, t, area(L, 1));
    hipLaunchKernelGGL(c_pcg_q, dim3(1), dim3(kBlock), 0, C->st, c, area(L, 1), nbi);
    hipLaunchKernelGGL((k_pcg_eigres<T>), dim3(nbi), dim3(kBlock), 0, C->st, n, c, u, Au, s_out, t, area(L, 2));
    const int seq = poll.next();
    hipLaunchKernelGGL(c_pcg_exit, dim3(1), dim3(kBlock), 0, C->st, c, area(L, 2), nbi, poll.flag(), seq);
    if (l > 0 && poll.read(seq - 1)) break;
  }
  DevCtl h = C->readctl();
  if (h.err) throw ApiError{BNX_E_BREAKDOWN, "triangular solve wait bound exceeded"};
  *its = h.its;
  *reason = h.reason;
}

// ------------------------------------------------------------------ double-precision helpers
// x <- x - Q (Q^T x) twice, then x <- x/||x||   (Q: nq columns, double)
void cgs2_normalize(bnx_ctx *C, double *x, double *tmp, int nq, const VList<double> &Q) {
  const Launch L = C->launch();
  DevCtl *c = C->ctl;
  const int n = C->n;
  VList<double> X{}, Y{};
  for (int q = 0; q < nq; q++) {
    X.p[q] = Q.p[q];
    Y.p[q] = x;
  }
  for (int pass = 0; pass < 2 && nq > 0; pass++) {
    int nb = launch_multidot<double, double>(L, n, nq, X, Y, area(L, 4), nullptr);
    hipLaunchKernelGGL(c_outer_cgs, dim3(1), dim3(kBlock), 0, C->st, c, area(L, 4), nb, nq, 0);
    comb<double>(C, tmp, x, 1.0, nullptr, nullptr, nullptr, nq, Q, c->oz, -1.0, 0, VList<double>{}, nullptr, nullptr);
    HIPCHK(hipMemcpyAsync(x, tmp, sizeof(double) * n, hipMemcpyDeviceToDevice, C->st));
  }
  VList<double> W = vl<double>({x});
  int nb = launch_multidot<double, double>(L, n, 1, W, W, area(L, 4), nullptr);
  hipLaunchKernelGGL(c_outer_cgs, dim3(1), dim3(kBlock), 0, C->st, c, area(L, 4), nb, 0, 1);
  hipLaunchKernelGGL(c_inv_sqrt, dim3(1), dim3(1), 0, C->st, c, &c->onrm2, &c->dinv);
  comb<double>(C, tmp, x, 1.0, &c->dinv, nullptr, nullptr, 0, VList<double>{}, nullptr, 0.0, 0, VList<double>{},
               nullptr, nullptr);
  HIPCHK(hipMemcpyAsync(x, tmp, sizeof(double) * n, hipMemcpyDeviceToDevice, C->st));
}

// Au = A u, theta = u^T A u, r = Au - theta u, ||r||; mirrors in T (when uT != nullptr)
template <typename T>
void outer_eval(bnx_ctx *C, const double *u, double *Au, double *r, T *uT, T *AuT, T *rT) {
  const Launch L = C->launch();
  DevCtl *c = C->ctl;
  const int n = C->n;
  Mat<double> A = C->mat<double>();
  VList<double> ly = vl<double>({u});
  int nb = launch_spmv<double>(L, A, u, Au, 1, ly, 0, VList<double>{}, area(L, 5), nullptr);
  hipLaunchKernelGGL(c_outer_theta, dim3(1), dim3(kBlock), 0, C->st, c, area(L, 5), nb);
  const int nbi = gridn(n);
  hipLaunchKernelGGL((k_outer_resid<T>), dim3(nbi), dim3(kBlock), 0, C->st, n, c, u, Au, r, uT, AuT, rT, area(L, 5));
  hipLaunchKernelGGL(c_outer_rn, dim3(1), dim3(kBlock), 0, C->st, c, area(L, 5), nbi);
}

// ------------------------------------------------------------------ DACG (Sec. 4.1)
// x (T) holds the normalised start vector; on return x is the DACG iterate (unit norm).  stall > 0
// also ends it after that many iterations without a 10 % gain near tol (*stalled is then set).
template <typename T>
int dacg(bnx_ctx *C, Work<T> &w, int nq, const VList<T> &Qt, double tol, int itmax, long long *mvp, int stall = 0,
         bool *stalled = nullptr) {
  const Launch L = C->launch();
  DevCtl *c = C->ctl;
  const int n = C->n;
  const int *gate = &c->ddone;
  Mat<T> A = C->mat<T>();
  Tri<T> Lf = C->tri<T>(true), Lt = C->tri<T>(false);
  const int nbi = gridn(n);
  hipLaunchKernelGGL(c_dacg_setup, dim3(1), dim3(64), 0, C->st, c, tol, itmax, stall);
  launch_fill<T>(C->st, n, w.d, T(0));  // no previous direction: the first step is d = -h
  // Ax
  launch_spmv<T>(L, A, w.x, w.Ax, 0, VList<T>{}, 0, VList<T>{}, nullptr, nullptr);
  (*mvp)++;
  VList<T> ly{}, lx{};
  ly.p[0] = w.d;
  lx.p[0] = w.Ax;
  lx.p[1] = w.x;
  lx.p[2] = w.d;
  // dots of the starting vector (no scaling: inv = 0)
  hipLaunchKernelGGL((k_dacg_scale<T>), dim3(nbi), dim3(kBlock), 0, C->st, n, c, w.x, w.Ax, area(L, 0));
  hipLaunchKernelGGL(c_dacg_q, dim3(1), dim3(kBlock), 0, C->st, c, area(L, 0), nbi);
  // the convergence test and the FP32 step's rescale run in the last block of their producers and reduce in
  // their own area, whose slots hold the empty mark between launches
  double *fa = area(L, kFusedArea);
  hipLaunchKernelGGL(k_arm, dim3(grid_for((size_t)kPartSlots * kNBMax, kNBMax)), dim3(kBlock), 0, C->st,
                     (unsigned long long *)fa, kPartSlots * kNBMax);
  Poll poll(C);
  // the first gradient (the start vector is already normalised: inv = 0 leaves it as it is) and the
  // convergence test of iteration 0; the FP64 test takes x^T x and x^T A x for the line search from it
  int seq = poll.next();
  hipLaunchKernelGGL((k_dacg_grad<T>), dim3(nbi), dim3(kBlock), 0, C->st, n, c, w.x, w.Ax, w.dg, fa, poll.flag(),
                     seq, sizeof(T) == 8 ? 1 : 0);
  int it;
  for (it = 0; it <= itmax; it++) {
    // h = (I - Qt Qt^T) P0^ g
    launch_trsv<T>(L, Lf, w.dg, w.z, 0, VList<T>{}, nullptr, gate);
    launch_trsv<T>(L, Lt, w.z, w.c0, 0, VList<T>{}, nullptr, gate);
    // one pass after the solves: Qt^T g, Qt^T c0, g^T c0
    int nbd = launch_mdot_list<T, T>(L, n, 2, w.dg, w.c0, nq, Qt, 1, area(L, 3), gate);
    hipLaunchKernelGGL(c_dacg_beta, dim3(1), dim3(kBlock), 0, C->st, c, area(L, 3), nbd, nq);
    // d = -(c0 - Qt zQ) + beta d
    // (dots of the new d with Ax, x and d itself)
    int nbc = comb<T>(C, w.d, w.c0, -1.0, nullptr, w.d, &c->beta, nq, Qt, c->zQ, 1.0, 3, lx, area(L, 9), gate);
    int nbs = launch_spmv<T>(L, A, w.d, w.Ad, 1, ly, 0, VList<T>{}, area(L, 4), gate);
    hipLaunchKernelGGL(c_dacg_alpha, dim3(1), dim3(kBlock), 0, C->st, c, area(L, 4), nbs, area(L, 9), nbc,
                       sizeof(T) == 8 ? 1 : 0);
    // the next iterate and gradient, with the convergence test of the next iteration
    const int nseq = poll.next();
    if constexpr (sizeof(T) == 8) {  // step, rescale and the next gradient in one pass
      hipLaunchKernelGGL(k_dacg_move, dim3(nbi), dim3(kBlock), 0, C->st, n, c, w.x, w.Ax, w.d, w.Ad, w.dg, fa,
                         poll.flag(), nseq);
    } else {
      hipLaunchKernelGGL((k_dacg_step<T>), dim3(nbi), dim3(kBlock), 0, C->st, n, c, w.x, w.Ax, w.d, w.Ad, fa);
      hipLaunchKernelGGL((k_dacg_grad<T>), dim3(nbi), dim3(kBlock), 0, C->st, n, c, w.x, w.Ax, w.dg, fa,
                         poll.flag(), nseq, 0);
    }
    // the test that gated the previous iteration: the device then still has about two iterations queued
    if (it > 0 && poll.read(seq - 1)) break;
    seq = nseq;
  }
  DevCtl h = C->readctl();
  if (h.err) throw ApiError{BNX_E_BREAKDOWN, "device wait bound exceeded (triangular solve or DACG reduction)"};
  // the last (gated) scale of x was skipped after convergence: x holds the scaled iterate
  *mvp += h.dits;
  if (stalled) *stalled = h.dstalled != 0;
  return h.dits;
}

// ------------------------------------------------------------------ Gram blocks from scratch
template <typename T>
void gram_full(bnx_ctx *C, int k, const VList<T> &S, const VList<T> &R, int m, const VList<T> &Q) {
  const Launch L = C->launch();
  const int n = C->n;
  if (k == 0) return;
  const int rows_per = kMaxVec / k;
  for (int kind = 0; kind < 2; kind++) {
    const int nrows_all = kind == 0 ? k : m;
    for (int r0 = 0; r0 < nrows_all; r0 += rows_per) {
      const int nr = std::min(rows_per, nrows_all - r0);
      VList<T> X{}, Y{};
      int D = 0;
      for (int a = 0; a < nr; a++)
        for (int t = 0; t < k; t++) {
          X.p[D] = kind == 0 ? S.p[r0 + a] : Q.p[r0 + a];
          Y.p[D++] = kind == 0 ? R.p[t] : S.p[t];
        }
      const int nb = launch_multidot<T, double>(L, n, D, X, Y, area(L, 6), nullptr);
      hipLaunchKernelGGL(c_gram_rows, dim3(1), dim3(kBlock), 0, C->st, C->ctl, area(L, 6), nb, k, kind, r0, nr);
    }
  }
}

// ------------------------------------------------------------------ splitmix64 start block
__global__ void k_splitmix(size_t count, uint64_t seed, double *out) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    out[i] = 2.0 * ((double)(z >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
  }
}

// ------------------------------------------------------------------ full solve (Alg. 2)
// x <- x - Q (Q^T x): one classical Gram-Schmidt pass (double)
void cgs_pass(bnx_ctx *C, double *x, double *tmp, int nq, const VList<double> &Q) {
  if (nq == 0) return;
  const Launch L = C->launch();
  DevCtl *c = C->ctl;
  VList<double> X{}, Y{};
  for (int q = 0; q < nq; q++) {
    X.p[q] = Q.p[q];
    Y.p[q] = x;
  }
  const int nb = launch_multidot<double, double>(L, C->n, nq, X, Y, area(L, 4), nullptr);
  hipLaunchKernelGGL(c_outer_cgs, dim3(1), dim3(kBlock), 0, C->st, c, area(L, 4), nb, nq, 0);
  comb<double>(C, tmp, x, 1.0, nullptr, nullptr, nullptr, nq, Q, c->oz, -1.0, 0, VList<double>{}, nullptr, nullptr);
  HIPCHK(hipMemcpyAsync(x, tmp, sizeof(double) * C->n, hipMemcpyDeviceToDevice, C->st));
}

// Jacobi-Davidson for eigenpair j (Sec. 6).  The search space V (orthonormal, orthogonal to the
// converged vectors Qt, at most mmax vectors; AV = A V kept beside it) starts from t.  Each step:
// expand V by t (classical Gram-Schmidt against Qt and V, twice), Rayleigh-Ritz on H = V^T A V,
// the smallest Ritz pair (theta, u) and r = A u - theta u, the outer test ||r|| <= tau theta, a
// thick restart with the mmin smallest Ritz vectors when V is full, then the correction s of
// J s = -r by the PCG of Sec. 4.3 with the BFGS pairs of the previous correction solves (kmax > 0).
// When the PCG takes no step (J indefinite far from the eigenvalue), V grows by the PCG's first
// preconditioned direction instead.  Leaves u, Au, r (double) of the last Ritz pair.
template <typename T>
void jd_pair(bnx_ctx *C, const bnx_solve_opts &o, Work<T> &w, int j, const VList<double> &Qt64, const VList<T> &QtT,
             double *t, double *u, double *Au, double *r, double *tmp, double *V, double *AV, double *Vt,
             bnx_stats &S, double &theta, double &rn, int &k) {
  const int n = C->n;
  const Launch L = C->launch();
  DevCtl *c = C->ctl;
  const bool fp64 = std::is_same<T, double>::value;
  const int mmax = o.jd_mmax, mmin = o.jd_mmin;
  Mat<double> A = C->mat<double>();
  T *uT = fp64 ? (T *)u : w.u, *AuT = fp64 ? (T *)Au : w.Au, *rT = fp64 ? (T *)r : w.r;
  std::deque<int> ring;
  bool inserted = false;
  int shift = 0, m = 0;
  k = 0;
  theta = rn = 0.0;
  for (;;) {
    // ---- expand V
    VList<double> VL{}, AVL{};
    for (int i = 0; i < m; i++) {
      VL.p[i] = V + (size_t)i * n;
      AVL.p[i] = AV + (size_t)i * n;
    }
    for (int pass = 0; pass < 2; pass++) {
      cgs_pass(C, t, tmp, j, Qt64);
      cgs_pass(C, t, tmp, m, VL);
    }
    VList<double> TT = vl<double>({t});
    int nb = launch_multidot<double, double>(L, n, 1, TT, TT, area(L, 4), nullptr);
    hipLaunchKernelGGL(c_outer_cgs, dim3(1), dim3(kBlock), 0, C->st, c, area(L, 4), nb, 0, 1);
    if (!(C->readctl().onrm2 > 0.0)) break;  // nothing left to add
    hipLaunchKernelGGL(c_inv_sqrt, dim3(1), dim3(1), 0, C->st, c, &c->onrm2, &c->dinv);
    double *vm = V + (size_t)m * n, *avm = AV + (size_t)m * n;
    comb<double>(C, vm, t, 1.0, &c->dinv, nullptr, nullptr, 0, VList<double>{}, nullptr, 0.0, 0, VList<double>{},
                 nullptr, nullptr);
    launch_spmv<double>(L, A, vm, avm, 0, VList<double>{}, 0, VList<double>{}, area(L, 5), nullptr);
    S.mvp_newton++;
    VL.p[m] = vm;
    AVL.p[m] = avm;
    VList<double> Y{};
    for (int i = 0; i <= m; i++) Y.p[i] = avm;
    nb = launch_multidot<double, double>(L, n, m + 1, VL, Y, area(L, 4), nullptr);
    hipLaunchKernelGGL(c_jd_col, dim3(1), dim3(kBlock), 0, C->st, c, area(L, 4), nb, m);
    m++;
    // ---- Rayleigh-Ritz: u = V y, A u = AV y for the smallest Ritz value, r = A u - theta u
    hipLaunchKernelGGL(c_jd_rr, dim3(1), dim3(64), 0, C->st, c, m);
    comb<double>(C, u, nullptr, 0.0, nullptr, nullptr, nullptr, m, VL, c->jY, 1.0, 0, VList<double>{}, nullptr,
                 nullptr);
    comb<double>(C, Au, nullptr, 0.0, nullptr, nullptr, nullptr, m, AVL, c->jY, 1.0, 0, VList<double>{}, nullptr,
                 nullptr);
    const int nbi = gridn(n);
    hipLaunchKernelGGL((k_outer_resid<T>), dim3(nbi), dim3(kBlock), 0, C->st, n, c, u, Au, r, fp64 ? nullptr : w.u,
                       fp64 ? nullptr : w.Au, fp64 ? nullptr : w.r, area(L, 5));
    hipLaunchKernelGGL(c_outer_rn, dim3(1), dim3(kBlock), 0, C->st, c, area(L, 5), nbi);
    // ---- Gram blocks of the pairs for this u (and for the pair stored after the last correction)
    const int kn = (int)ring.size();
    if (kn > 0) {
      VList<T> X{}, Yg{};
      int D = 0;
      if (inserted) {
        const T *snew = w.S[ring.back()], *rnew = w.R[ring.back()];
        for (int q = 0; q < kn; q++) {
          X.p[D] = snew;
          Yg.p[D++] = w.R[ring[q]];
        }
        for (int q = 0; q < kn - 1; q++) {
          X.p[D] = w.S[ring[q]];
          Yg.p[D++] = rnew;
        }
        for (int q = 0; q < j; q++) {
          X.p[D] = QtT.p[q];
          Yg.p[D++] = snew;
        }
      }
      for (int q = 0; q < kn; q++) {
        X.p[D] = uT;
        Yg.p[D++] = w.S[ring[q]];
      }
      const int nbg = launch_multidot<T, double>(L, n, D, X, Yg, area(L, 6), nullptr);
      hipLaunchKernelGGL(c_gram, dim3(1), dim3(kBlock), 0, C->st, c, area(L, 6), nbg, shift, inserted ? 1 : 0, kn,
                         j);
    }
    inserted = false;
    shift = 0;
    const DevCtl h = C->readctl();
    theta = h.otheta;
    rn = h.orn;
    if (rn <= o.tol * theta || k >= o.itmax) break;
    if (m == mmax) {  // thick restart: the mmin smallest Ritz vectors (u is the first)
      for (int cc = 0; cc < mmin; cc++)
        comb<double>(C, Vt + (size_t)cc * n, nullptr, 0.0, nullptr, nullptr, nullptr, m, VL, c->jY + cc * kJdMax,
                     1.0, 0, VList<double>{}, nullptr, nullptr);
      HIPCHK(hipMemcpyAsync(V, Vt, sizeof(double) * n * mmin, hipMemcpyDeviceToDevice, C->st));
      for (int cc = 0; cc < mmin; cc++)
        comb<double>(C, Vt + (size_t)cc * n, nullptr, 0.0, nullptr, nullptr, nullptr, m, AVL, c->jY + cc * kJdMax,
                     1.0, 0, VList<double>{}, nullptr, nullptr);
      HIPCHK(hipMemcpyAsync(AV, Vt, sizeof(double) * n * mmin, hipMemcpyDeviceToDevice, C->st));
      hipLaunchKernelGGL(c_jd_restart, dim3(1), dim3(64), 0, C->st, c, mmin);
      m = mmin;
    }
    // ---- correction equation
    VList<T> Q = QtT;
    Q.p[j] = uT;
    VList<T> AQ{};
    for (int q = 0; q < j; q++) AQ.p[q] = w.AQm + (size_t)q * n;
    AQ.p[j] = AuT;
    VList<T> SL{}, RL{};
    for (size_t q = 0; q < ring.size(); q++) {
      SL.p[q] = w.S[ring[q]];
      RL.p[q] = w.R[ring[q]];
    }
    PcgParams P;
    P.theta = theta;
    P.tol_pcg = o.tol_pcg;
    P.itmax = o.itmax_pcg;
    P.tau = o.tol;
    P.exit_rule = o.exit_rule;
    P.xi = o.exit_xi;
    P.sgn = -1.0;
    P.eigtest = 1;
    int its = 0, why = 0;
    pcg<T>(C, w, P, rT, j + 1, Q, AQ, (int)ring.size(), SL, RL, uT, AuT, w.s, &its, &why);
    S.pcg_its[j] += its;
    S.mvp_newton += its;
    if (why == 4) S.pcg_breakdowns++;
    if (its > 0) {
      // the pair (s_k, r_k) of Alg. 2, stored unless s^T r >= -1e-12 ||s|| ||r||
      VList<T> X{}, Yd{};
      X.p[0] = w.s;
      Yd.p[0] = rT;
      X.p[1] = w.s;
      Yd.p[1] = w.s;
      const int nb2 = launch_multidot<T, double>(L, n, 2, X, Yd, area(L, 4), nullptr);
      hipLaunchKernelGGL(c_outer_y, dim3(1), dim3(kBlock), 0, C->st, c, area(L, 4), nb2);
      const DevCtl hy = C->readctl();
      if (o.kmax > 0 && hy.oya < -1e-12 * std::sqrt(hy.oyn2) * rn) {
        int slot;
        if ((int)ring.size() == o.kmax) {
          slot = ring.front();
          ring.pop_front();
          shift = 1;
        } else {
          std::vector<bool> used(o.kmax, false);
          for (int q : ring) used[q] = true;
          slot = 0;
          while (used[slot]) slot++;
        }
        HIPCHK(hipMemcpyAsync(w.S[slot], w.s, sizeof(T) * n, hipMemcpyDeviceToDevice, C->st));
        launch_cast<double, T>(C->st, n, r, w.R[slot]);
        ring.push_back(slot);
        inserted = true;
      } else {
        S.bfgs_skipped++;
      }
      launch_cast<T, double>(C->st, n, w.s, t);
    } else {
      launch_cast<T, double>(C->st, n, w.p, t);  // the first preconditioned direction
    }
    k++;
  }
}

template <typename T>
bnx_status solve_impl(bnx_ctx *C, const bnx_solve_opts &o, double *evals, double *evecs, bnx_stats *st) {
  const int n = C->n, p = o.p;
  const Launch L = C->launch();
  DevCtl *c = C->ctl;
  const bool fp64 = std::is_same<T, double>::value;
  Work<T> w;
  make_work<T>(C, w, o.kmax, p);
  std::unique_ptr<Work<double>> w64;  // double DACG for stall restarts of the mixed path
  struct Guard {
    bnx_ctx *C;
    Work<T> *w;
    std::unique_ptr<Work<double>> *w64;
    std::vector<double *> extra;
    ~Guard() {
      free_work<T>(C, *w);
      if (*w64) free_work<double>(C, **w64);
      for (double *q : extra) C->release(q);
    }
  } guard{C, &w, &w64, {}};
  auto dalloc = [&](size_t cnt) {
    double *q = C->alloc<double>(cnt);
    guard.extra.push_back(q);
    return q;
  };
  double *V64 = dalloc((size_t)n * p);  // converged vectors v_1..v_p (unsorted)
  double *X0 = dalloc((size_t)n * p);
  double *u = dalloc(n), *Au = dalloc(n), *rA = dalloc(n), *rB = dalloc(n), *x64 = dalloc(n), *tmp = dalloc(n);
  double *Vjd = nullptr, *AVjd = nullptr, *Vtjd = nullptr;  // Jacobi-Davidson search space
  if (o.jd) {
    Vjd = dalloc((size_t)n * o.jd_mmax);
    AVjd = dalloc((size_t)n * o.jd_mmax);
    Vtjd = dalloc((size_t)n * o.jd_mmin);
  }
  if (o.x0) {
    HIPCHK(hipMemcpyAsync(X0, o.x0, sizeof(double) * n * p, C->device_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                          C->st));
  } else {
    hipLaunchKernelGGL(k_splitmix, dim3(1024), dim3(kBlock), 0, C->st, (size_t)n * p, (uint64_t)o.seed, X0);
  }
  std::vector<double> lam(p);
  bnx_stats S{};
  double t0;
  for (int j = 0; j < p; j++) {
    // ---- start vector orthogonal to v_1..v_{j-1} and DACG (Sec. 4.1)
    t0 = now_s();
    VList<double> Qt64{};
    VList<T> QtT{};
    for (int q = 0; q < j; q++) {
      Qt64.p[q] = V64 + (size_t)q * n;
      QtT.p[q] = fp64 ? (const T *)(V64 + (size_t)q * n) : w.Qm + (size_t)q * n;
    }
    HIPCHK(hipMemcpyAsync(x64, X0 + (size_t)j * n, sizeof(double) * n, hipMemcpyDeviceToDevice, C->st));
    cgs2_normalize(C, x64, tmp, j, Qt64);
    if (o.jd) {  // Jacobi-Davidson from the start vector, no DACG (Sec. 6)
      t0 = now_s();
      double theta_j = 0.0, rn_j = 0.0;
      int k_j = 0;
      jd_pair<T>(C, o, w, j, Qt64, QtT, x64, u, Au, rA, tmp, Vjd, AVjd, Vtjd, S, theta_j, rn_j, k_j);
      S.outer_its[j] = k_j;
      S.relres[j] = rn_j / theta_j;
      S.converged[j] = rn_j <= o.tol * theta_j;
      lam[j] = theta_j;
      HIPCHK(hipMemcpyAsync(V64 + (size_t)j * n, u, sizeof(double) * n, hipMemcpyDeviceToDevice, C->st));
      if (!fp64) launch_cast<double, T>(C->st, n, u, w.Qm + (size_t)j * n);
      launch_cast<double, T>(C->st, n, Au, w.AQm + (size_t)j * n);
      C->sync();
      S.t_newton += now_s() - t0;
      continue;
    }
    launch_cast<double, T>(C->st, n, x64, w.x);
    long long mvp = 0;
    // DACG to tau_DACG before Newton; alone, to the final tau, and then always in double (tau is far
    // below the float residual floor)
    const bool alone = o.newton == 0;
    if (alone && !fp64) {
      if (!w64) {
        w64.reset(new Work<double>);
        make_work<double>(C, *w64, 0, 0);
      }
      HIPCHK(hipMemcpyAsync(w64->x, x64, sizeof(double) * n, hipMemcpyDeviceToDevice, C->st));
      S.dacg_its[j] = dacg<double>(C, *w64, j, Qt64, o.tol, o.itmax_dacg, &mvp);
      HIPCHK(hipMemcpyAsync(u, w64->x, sizeof(double) * n, hipMemcpyDeviceToDevice, C->st));
    } else {
      bool stalled = false;
      S.dacg_its[j] = dacg<T>(C, w, j, QtT, alone ? o.tol : o.tol_dacg, o.itmax_dacg, &mvp, fp64 ? 0 : kDacgStall,
                              &stalled);
      launch_cast<T, double>(C->st, n, w.x, u);
      if (stalled) {
        // the float iterate stopped gaining at its residual floor, above tau_DACG q: the double
        // DACG takes it from there to tau_DACG
        if (!w64) {
          w64.reset(new Work<double>);
          make_work<double>(C, *w64, 0, 0);
        }
        cgs2_normalize(C, u, tmp, j, Qt64);
        HIPCHK(hipMemcpyAsync(w64->x, u, sizeof(double) * n, hipMemcpyDeviceToDevice, C->st));
        S.dacg_its[j] += dacg<double>(C, *w64, j, Qt64, o.tol_dacg, std::max(0, o.itmax_dacg - S.dacg_its[j]), &mvp);
        HIPCHK(hipMemcpyAsync(u, w64->x, sizeof(double) * n, hipMemcpyDeviceToDevice, C->st));
      }
    }
    S.mvp_dacg += mvp;
    C->sync();
    S.t_dacg += now_s() - t0;

    // ---- Newton phase
    t0 = now_s();
    cgs2_normalize(C, u, tmp, j, Qt64);
    double *r_old = rA, *r_new = rB;
    T *uT = fp64 ? (T *)u : w.u, *AuT = fp64 ? (T *)Au : w.Au, *rT = fp64 ? (T *)r_old : w.r;
    outer_eval<T>(C, u, Au, r_old, fp64 ? nullptr : w.u, fp64 ? nullptr : w.Au, fp64 ? nullptr : w.r);
    S.mvp_newton++;
    DevCtl h = C->readctl();
    double theta = h.otheta, rn = h.orn;
    std::deque<int> ring;  // chronological slots
    int k = 0, slow = 0, restarts = 0;
    double t_restart = 0.0;  // DACG time inside the Newton phase: counted in t_dacg only
    double best = rn;  // mixed precision: smallest outer residual so far
    int since_best = 0;

    while (!alone && rn > o.tol * theta && k < o.itmax) {
      const int m = j + 1;
      VList<T> Q = QtT;
      Q.p[j] = uT;
      VList<T> SL{}, RL{};
      for (size_t t = 0; t < ring.size(); t++) {
        SL.p[t] = w.S[ring[t]];
        RL.p[t] = w.R[ring[t]];
      }
      const int kk = (int)ring.size();
      PcgParams P;
      P.theta = theta;
      P.tol_pcg = o.tol_pcg;
      P.itmax = o.itmax_pcg;
      P.tau = o.tol;
      P.exit_rule = o.exit_rule;
      P.xi = o.exit_xi;
      P.sgn = -1.0;
      P.eigtest = 1;
      int its = 0, why = 0;
      rT = fp64 ? (T *)r_old : w.r;
      VList<T> AQ{};
      for (int q = 0; q < j; q++) AQ.p[q] = w.AQm + (size_t)q * n;
      AQ.p[j] = AuT;
      pcg<T>(C, w, P, rT, m, Q, AQ, kk, SL, RL, uT, AuT, w.s, &its, &why);
      S.pcg_its[j] += its;
      S.mvp_newton += its;
      if (why == 4) S.pcg_breakdowns++;
      // ---- outer step: u <- (u + s)/||u + s||, re-orthogonalised against v_1..v_{j-1} (double)
      const int nbi = gridn(n);
      if (3 + j <= 8)
        hipLaunchKernelGGL((k_outer_add<T, 8>), dim3(nbi), dim3(kBlock), 0, C->st, n, u, w.s, r_old, x64, j, Qt64,
                           area(L, 4));
      else if (3 + j <= 16)
        hipLaunchKernelGGL((k_outer_add<T, 16>), dim3(nbi), dim3(kBlock), 0, C->st, n, u, w.s, r_old, x64, j, Qt64,
                           area(L, 4));
      else
        hipLaunchKernelGGL((k_outer_add<T, 3 + kMaxQ>), dim3(nbi), dim3(kBlock), 0, C->st, n, u, w.s, r_old, x64, j,
                           Qt64, area(L, 4));
      hipLaunchKernelGGL(c_outer_add, dim3(1), dim3(kBlock), 0, C->st, c, area(L, 4), nbi, j);
      hipLaunchKernelGGL(c_inv_sqrt, dim3(1), dim3(1), 0, C->st, c, &c->onrm2, &c->dinv);
      comb<double>(C, u, x64, 1.0, &c->dinv, nullptr, nullptr, 0, VList<double>{}, nullptr, 0.0, 0, VList<double>{},
                   nullptr, nullptr);
      cgs2_normalize(C, u, tmp, j, Qt64);
      outer_eval<T>(C, u, Au, r_new, fp64 ? nullptr : w.u, fp64 ? nullptr : w.Au, fp64 ? nullptr : w.r);
      S.mvp_newton++;
      h = C->readctl();
      const double alpha = h.oalpha, sn2 = h.osn2;
      // ---- store the pair in the k_max window (Sec. 4.4): (s_k, r_k), or with the full update of eq. (2.1)
      //      (s_k, r_k - r_{k+1}); either way alpha = s^T(stored) < 0 keeps the preconditioner SPD
      bool insert;
      if (o.bfgs_full) {
        const int nbi2 = gridn(n);
        hipLaunchKernelGGL((k_ydiff<T>), dim3(nbi2), dim3(kBlock), 0, C->st, n, r_old, r_new, w.z);
        VList<T> X{}, Y{};
        X.p[0] = w.s;
        Y.p[0] = w.z;
        X.p[1] = w.z;
        Y.p[1] = w.z;
        const int nb2 = launch_multidot<T, double>(L, n, 2, X, Y, area(L, 4), nullptr);
        hipLaunchKernelGGL(c_outer_y, dim3(1), dim3(kBlock), 0, C->st, c, area(L, 4), nb2);
        const DevCtl hy = C->readctl();
        insert = o.kmax > 0 && hy.oya < -1e-12 * std::sqrt(sn2) * std::sqrt(hy.oyn2);
      } else {
        insert = o.kmax > 0 && alpha < -1e-12 * std::sqrt(sn2) * rn;
      }
      int shift = 0;
      if (insert) {
        int slot;
        if ((int)ring.size() == o.kmax) {
          slot = ring.front();
          ring.pop_front();
          shift = 1;
        } else {
          slot = (int)ring.size();
          // the first free slot: slots are used 0..kmax-1 before any reuse
          std::vector<bool> used(o.kmax, false);
          for (int q : ring) used[q] = true;
          for (int q = 0; q < o.kmax; q++)
            if (!used[q]) {
              slot = q;
              break;
            }
        }
        HIPCHK(hipMemcpyAsync(w.S[slot], w.s, sizeof(T) * n, hipMemcpyDeviceToDevice, C->st));
        if (o.bfgs_full) HIPCHK(hipMemcpyAsync(w.R[slot], w.z, sizeof(T) * n, hipMemcpyDeviceToDevice, C->st));
        else launch_cast<double, T>(C->st, n, r_old, w.R[slot]);
        ring.push_back(slot);
      } else {
        S.bfgs_skipped++;
      }
      // ---- Gram blocks (double): new row/column of M, Qt^T s_new, and u^T S for the new u
      const int kn = (int)ring.size();
      if (kn > 0) {
        VList<T> X{}, Y{};
        int D = 0;
        if (insert) {
          const T *snew = w.S[ring.back()], *rnew = w.R[ring.back()];
          for (int t = 0; t < kn; t++) {
            X.p[D] = snew;
            Y.p[D++] = w.R[ring[t]];
          }
          for (int t = 0; t < kn - 1; t++) {
            X.p[D] = w.S[ring[t]];
            Y.p[D++] = rnew;
          }
          for (int q = 0; q < j; q++) {
            X.p[D] = QtT.p[q];
            Y.p[D++] = snew;
          }
        }
        for (int t = 0; t < kn; t++) {
          X.p[D] = uT;
          Y.p[D++] = w.S[ring[t]];
        }
        int nb = launch_multidot<T, double>(L, n, D, X, Y, area(L, 6), nullptr);
        hipLaunchKernelGGL(c_gram, dim3(1), dim3(kBlock), 0, C->st, c, area(L, 6), nb, shift, insert ? 1 : 0, kn, j);
      }
      std::swap(r_old, r_new);
      // stall: no PCG step, or the residual fails to drop below 0.9x twice in a row
      slow = (its == 0 || h.orn > 0.9 * rn) ? slow + 1 : 0;
      theta = h.otheta;
      rn = h.orn;
      k++;
      // Mixed precision: the float inner solves bound how far the outer residual can fall.  When
      // it is below 1e-7 theta (float territory) and has not improved on its best by 10 % for
      // three steps (it oscillates at that floor rather than stalling), the pair is finished by
      // the double DACG to tau.
      if (rn < 0.9 * best) {
        best = rn;
        since_best = 0;
      } else {
        since_best++;
      }
      const bool floor = !fp64 && since_best >= 3 && rn < 1e-7 * theta;
      if ((its == 0 || slow >= 2 || floor) && restarts < 5 && rn > o.tol * theta && k < o.itmax) {
        // the start was not close enough (Sec. 4.1): resume DACG from u with a tighter tolerance,
        // restart the BFGS history, then continue Newton
        const double td2 = now_s();
        const double t2 = floor ? o.tol : std::min(o.tol_dacg, std::max(o.tol, 0.005 * rn / theta));
        long long mvp2 = 0;
        if (fp64) {
          launch_cast<double, T>(C->st, n, u, w.x);
          S.dacg_its[j] += dacg<T>(C, w, j, QtT, t2, o.itmax_dacg, &mvp2);
          launch_cast<T, double>(C->st, n, w.x, u);
        } else {
          // tolerances below the float residual floor need the double DACG
          if (!w64) {
            w64.reset(new Work<double>);
            make_work<double>(C, *w64, 0, 0);
          }
          HIPCHK(hipMemcpyAsync(w64->x, u, sizeof(double) * n, hipMemcpyDeviceToDevice, C->st));
          S.dacg_its[j] += dacg<double>(C, *w64, j, Qt64, t2, o.itmax_dacg, &mvp2);
          HIPCHK(hipMemcpyAsync(u, w64->x, sizeof(double) * n, hipMemcpyDeviceToDevice, C->st));
        }
        S.mvp_dacg += mvp2;
        cgs2_normalize(C, u, tmp, j, Qt64);
        ring.clear();
        outer_eval<T>(C, u, Au, r_old, fp64 ? nullptr : w.u, fp64 ? nullptr : w.Au, fp64 ? nullptr : w.r);
        S.mvp_newton++;
        h = C->readctl();
        theta = h.otheta;
        rn = h.orn;
        restarts++;
        S.dacg_restarts++;
        slow = 0;
        best = rn;
        since_best = 0;
        const double dt2 = now_s() - td2;
        S.t_dacg += dt2;
        t_restart += dt2;
      }
    }
    S.outer_its[j] = k;
    S.relres[j] = rn / theta;
    S.converged[j] = rn <= o.tol * theta;
    lam[j] = theta;
    HIPCHK(hipMemcpyAsync(V64 + (size_t)j * n, u, sizeof(double) * n, hipMemcpyDeviceToDevice, C->st));
    if (!fp64) launch_cast<double, T>(C->st, n, u, w.Qm + (size_t)j * n);
    launch_cast<double, T>(C->st, n, Au, w.AQm + (size_t)j * n);  // A v_j from the last outer step
    C->sync();
    S.t_newton += now_s() - t0 - t_restart;
  }
  // ---- sort ascending, fix signs, write outputs
  std::vector<int> idx(p);
  for (int j = 0; j < p; j++) idx[j] = j;
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return lam[a] < lam[b]; });
  if (C->evecs_last) C->release(C->evecs_last);
  C->evecs_last = C->alloc<double>((size_t)n * p);
  double *pm = area(L, 7), *pi = area(L, 7) + kNBMax;
  for (int jj = 0; jj < p; jj++) {
    const double *v = V64 + (size_t)idx[jj] * n;
    const int nb = gridn(n);
    hipLaunchKernelGGL(k_absmax, dim3(nb), dim3(kBlock), 0, C->st, n, v, pm);
    hipLaunchKernelGGL(k_firstbig, dim3(nb), dim3(kBlock), 0, C->st, n, v, pm, nb, pi);
    hipLaunchKernelGGL(k_sign_copy, dim3(nb), dim3(kBlock), 0, C->st, n, v, pi, nb, C->evecs_last + (size_t)jj * n);
  }
  bnx_stats So = S;
  for (int jj = 0; jj < p; jj++) {
    evals[jj] = lam[idx[jj]];
    So.dacg_its[jj] = S.dacg_its[idx[jj]];
    So.outer_its[jj] = S.outer_its[idx[jj]];
    So.pcg_its[jj] = S.pcg_its[idx[jj]];
    So.relres[jj] = S.relres[idx[jj]];
    So.converged[jj] = S.converged[idx[jj]];
  }
  if (evecs)
    HIPCHK(hipMemcpyAsync(evecs, C->evecs_last, sizeof(double) * n * p,
                          C->device_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, C->st));
  C->sync();
  C->evals_last.assign(evals, evals + p);
  C->p_last = p;
  C->prec_last = fp64 ? BNX_FP64 : BNX_MIXED;
  C->solved = true;
  bool allc = true;
  for (int jj = 0; jj < p; jj++) allc = allc && So.converged[jj];
  So.status = allc ? BNX_OK : BNX_NOT_CONVERGED;
  const Analysis &run_an = (C->lps && !fp64) ? C->anS : *C->ta;  // the systems this solve's substitutions ran
  So.levels_L = run_an.levL.nlev;
  So.levels_Lt = run_an.levLt.nlev;
  So.nnz_L = C->ta->nnzL;
  So.fill = (double)C->ta->nnzL / (double)C->an.nnzL;
  So.shift_used = C->shift_used;
  So.t_factor = C->t_factor;
  if (st) *st = So;
  return (bnx_status)So.status;
}

// ------------------------------------------------------------------ backward
// out = (I - QQ^T) x  (double, CGS twice), out != x
void project_out(bnx_ctx *C, double *out, const double *x, int m, const VList<double> &Q, double *tmp) {
  const Launch L = C->launch();
  const int n = C->n;
  DevCtl *c = C->ctl;
  HIPCHK(hipMemcpyAsync(out, x, sizeof(double) * n, hipMemcpyDeviceToDevice, C->st));
  VList<double> X{}, Y{};
  for (int q = 0; q < m; q++) {
    X.p[q] = Q.p[q];
    Y.p[q] = out;
  }
  for (int pass = 0; pass < 2; pass++) {
    const int nb = launch_multidot<double, double>(L, n, m, X, Y, area(L, 6), nullptr);
    hipLaunchKernelGGL(c_outer_cgs, dim3(1), dim3(kBlock), 0, C->st, c, area(L, 6), nb, m, 0);
    comb<double>(C, tmp, out, 1.0, nullptr, nullptr, nullptr, m, Q, c->oz, -1.0, 0, VList<double>{}, nullptr, nullptr);
    HIPCHK(hipMemcpyAsync(out, tmp, sizeof(double) * n, hipMemcpyDeviceToDevice, C->st));
  }
}

double norm2_host(bnx_ctx *C, const double *x) {
  const Launch L = C->launch();
  VList<double> X = vl<double>({x});
  const int nb = launch_multidot<double, double>(L, C->n, 1, X, X, area(L, 6), nullptr);
  hipLaunchKernelGGL(c_reduce_to, dim3(1), dim3(kBlock), 0, C->st, C->ctl->bz, area(L, 6), nb, 1);
  return std::sqrt(C->readctl().bz[0]);
}

// Returns an empty string, or a description of the adjoint solves that missed tol_adj.
template <typename T>
std::string backward_impl(bnx_ctx *C, const double *g_evals, const double *g_evecs_dev, double *gv) {
  const int n = C->n, p = C->p_last;
  const Launch L = C->launch();
  DevCtl *c = C->ctl;
  const bool fp64 = std::is_same<T, double>::value;
  const double *V = C->evecs_last;
  Work<T> w;
  make_work<T>(C, w, 0, p);
  struct Guard {
    bnx_ctx *C;
    Work<T> *w;
    std::vector<double *> extra;
    ~Guard() {
      free_work<T>(C, *w);
      for (double *q : extra) C->release(q);
    }
  } guard{C, &w, {}};
  auto dalloc = [&](size_t cnt) {
    double *q = C->alloc<double>(cnt);
    guard.extra.push_back(q);
    return q;
  };
  double *ge = dalloc(p), *lam = dalloc(p), *xi = dalloc(n), *eta = dalloc(n), *res = dalloc(n), *tmp = dalloc(n);
  double *Ae = dalloc(n), *rhs = dalloc(n), *tmp2 = dalloc(n), *scal = dalloc(4);
  HIPCHK(hipMemcpyAsync(ge, g_evals, sizeof(double) * p, hipMemcpyHostToDevice, C->st));
  HIPCHK(hipMemcpyAsync(lam, C->evals_last.data(), sizeof(double) * p, hipMemcpyHostToDevice, C->st));
  HIPCHK(hipMemsetAsync(&c->err, 0, sizeof(int), C->st));
  launch_fill<double>(C->st, C->nnz, gv, 0.0);
  // sum_i g_evals[i] v_i v_i^T on the pattern
  hipLaunchKernelGGL(k_grad_lambda, dim3(gridn(n)), dim3(kBlock), 0, C->st, n, C->rp, C->ci, p, V, ge, gv);
  if (!g_evecs_dev) {
    C->sync();
    return std::string();
  }
  std::string missed;
  if (!fp64)
    for (int q = 0; q < p; q++) launch_cast<double, T>(C->st, n, V + (size_t)q * n, w.Qm + (size_t)q * n);
  Mat<double> A64 = C->mat<double>();
  for (int q = 0; q < p; q++) {  // A v_q for the projection coefficients of the adjoint PCG
    launch_spmv<double>(L, A64, V + (size_t)q * n, tmp, 0, VList<double>{}, 0, VList<double>{}, nullptr, nullptr);
    launch_cast<double, T>(C->st, n, tmp, w.AQm + (size_t)q * n);
  }
  for (int i = 0; i < p; i++) {
    const double *G = g_evecs_dev + (size_t)i * n;
    if (!(norm2_host(C, G) > 0.0)) continue;
    const int m = i + 1;
    VList<double> Vl{};
    for (int j = 0; j < m; j++) Vl.p[j] = V + (size_t)j * n;
    // explicit part along v_j, j < i: xi = sum_j v_j (v_j^T G)/(lambda_j - lambda_i)
    if (i > 0) {
      VList<double> Gl{};
      for (int j = 0; j < i; j++) Gl.p[j] = G;
      const int nb = launch_multidot<double, double>(L, n, i, Vl, Gl, area(L, 6), nullptr);
      hipLaunchKernelGGL(c_adj_coef, dim3(1), dim3(kBlock), 0, C->st, c, area(L, 6), nb, i, lam, i);
      comb<double>(C, xi, nullptr, 0.0, nullptr, nullptr, nullptr, i, Vl, c->bz, 1.0, 0, VList<double>{}, nullptr,
                   nullptr);
    } else {
      launch_fill<double>(C->st, n, xi, 0.0);
    }
    // eta in the complement of Q = [v_1..v_i]: (I-QQ^T)(A - lambda_i I)(I-QQ^T) eta = (I-QQ^T) G
    VList<T> Q{}, AQ{};
    for (int q = 0; q < m; q++) {
      Q.p[q] = fp64 ? (const T *)(V + (size_t)q * n) : w.Qm + (size_t)q * n;
      AQ.p[q] = w.AQm + (size_t)q * n;
    }
    project_out(C, rhs, G, m, Vl, tmp);
    const double rhs_n = norm2_host(C, rhs);
    launch_fill<double>(C->st, n, eta, 0.0);
    HIPCHK(hipMemcpyAsync(res, rhs, sizeof(double) * n, hipMemcpyDeviceToDevice, C->st));
    PcgParams P;
    P.theta = C->evals_last[i];
    P.itmax = C->adj_itmax;
    P.tau = 0.0;
    P.exit_rule = 0;
    P.eigtest = 0;
    P.sgn = 1.0;
    // res = rhs - (I-QQ^T)(A eta - lambda eta) in double; returns ||res||
    auto true_residual = [&]() {
      launch_spmv<double>(L, A64, eta, Ae, 0, VList<double>{}, 0, VList<double>{}, nullptr, nullptr);
      hipLaunchKernelGGL(c_set, dim3(1), dim3(1), 0, C->st, scal + 1, -C->evals_last[i]);
      comb<double>(C, tmp, Ae, 1.0, nullptr, eta, scal + 1, 0, VList<double>{}, nullptr, 0.0, 0, VList<double>{},
                   nullptr, nullptr);
      project_out(C, tmp2, tmp, m, Vl, Ae);
      hipLaunchKernelGGL(c_set, dim3(1), dim3(1), 0, C->st, scal + 2, -1.0);
      comb<double>(C, res, rhs, 1.0, nullptr, tmp2, scal + 2, 0, VList<double>{}, nullptr, 0.0, 0, VList<double>{},
                   nullptr, nullptr);
      return norm2_host(C, res);
    };
    bool ok = true;
    double resn = rhs_n;
    if (fp64) {
      P.tol_pcg = C->adj_tol;
      int its = 0, why = 0;
      pcg<T>(C, w, P, (const T *)res, m, Q, AQ, 0, VList<T>{}, VList<T>{}, nullptr, nullptr, (T *)eta, &its, &why);
      // reason 1: the recurred residual met tol_adj.  After the cap or a breakdown (p^T J p <= 0, which
      // rounding produces once the residual is at its floor) the true residual decides.
      if (why != 1) {
        resn = true_residual();
        ok = resn <= C->adj_tol * rhs_n;
      }
    } else {
      // float PCG inside double iterative refinement
      P.tol_pcg = 1e-4;
      for (int round = 0; round < 40 && resn > C->adj_tol * rhs_n; round++) {
        launch_cast<double, T>(C->st, n, res, w.r);
        int its = 0, why = 0;
        pcg<T>(C, w, P, w.r, m, Q, AQ, 0, VList<T>{}, VList<T>{}, nullptr, nullptr, w.s, &its, &why);
        launch_cast<T, double>(C->st, n, w.s, tmp);
        // eta += delta  (coefficient 1 via scal[0])
        hipLaunchKernelGGL(c_set, dim3(1), dim3(1), 0, C->st, scal, 1.0);
        comb<double>(C, tmp2, eta, 1.0, nullptr, tmp, scal, 0, VList<double>{}, nullptr, 0.0, 0, VList<double>{},
                     nullptr, nullptr);
        HIPCHK(hipMemcpyAsync(eta, tmp2, sizeof(double) * n, hipMemcpyDeviceToDevice, C->st));
        resn = true_residual();
      }
      ok = resn <= C->adj_tol * rhs_n;
    }
    if (!ok) {
      char buf[160];
      snprintf(buf, sizeof buf, "%sadjoint solve of pair %d: residual %.3g > tol_adj %.3g (relative)",
               missed.empty() ? "" : "; ", i + 1, resn / rhs_n, C->adj_tol);
      missed += buf;
    }
    // xi += eta; g_vals -= 1/2 (xi v_i^T + v_i xi^T) on the pattern
    hipLaunchKernelGGL(c_set, dim3(1), dim3(1), 0, C->st, scal + 3, 1.0);
    comb<double>(C, tmp, xi, 1.0, nullptr, eta, scal + 3, 0, VList<double>{}, nullptr, 0.0, 0, VList<double>{}, nullptr,
                 nullptr);
    hipLaunchKernelGGL(k_grad_vec, dim3(gridn(n)), dim3(kBlock), 0, C->st, n, C->rp, C->ci, V + (size_t)i * n, tmp, gv);
  }
  DevCtl h = C->readctl();
  if (h.err) throw ApiError{BNX_E_BREAKDOWN, "triangular solve wait bound exceeded"};
  return missed;
}

// ------------------------------------------------------------------ factor
// Device copy of a triangular pattern (rows of L and of L^T, level sets) and the
// LDS block schedules of its two solves, replacing whatever pattern was there.
// Values are filled in by the factorisation.
void build_tri(bnx_ctx *C, const Analysis &a) {
  C->sync();
  for (int dir = 0; dir < 2; dir++)
    for (int pr = 0; pr < 2; pr++) {
      auto &b = C->blk[dir][pr];
      for (int *q : {b.bptr, b.brows, b.iptr, b.isrc, b.eptr, b.erank, b.orow, b.oslot, b.perm, b.slice_ptr,
                     b.slice_nnz, b.ref, b.valmap, b.diagmap, b.cnt, b.ref4, b.valmap4, b.mjr, b.mtr})
        C->release(q);
      for (double *q : {b.diag64, b.val64, b.val4_64}) C->release(q);
      for (float *q : {b.diag32, b.val32, b.val4_32}) C->release(q);
      b = bnx_ctx::BlkDev{};
    }
  for (int *q : {C->Lrp, C->Lci, C->mapL, C->Ltrp, C->Ltci, C->mapLt, C->levL, C->levLt}) C->release(q);
  for (double *q : {C->Lv, C->Ltv, C->blk_exp64}) C->release(q);
  for (float *q : {C->Lv32, C->Ltv32, C->blk_exp32}) C->release(q);
  C->release(C->blk_cnt);
  C->blk_exp64 = nullptr;
  C->blk_exp32 = nullptr;
  C->blk_cnt = nullptr;
  for (auto &S : C->sys) {
    for (int *q : {S.rp, S.ci, S.lev, S.direct, S.tp, S.ta, S.tb, S.tc, S.mp, S.mj, S.ma, S.mc}) C->release(q);
    for (double *q : {S.v, S.mv}) C->release(q);
    for (float *q : {S.v32, S.mv32}) C->release(q);
    S = bnx_ctx::SysDev{};
  }
  C->lps = false;
  C->ta = nullptr;
  C->factored = false;
  C->solved = false;
  const int n = a.n;
  const int nnzL = a.nnzL;
  C->Lrp = C->alloc<int>(n + 1);
  C->Lci = C->alloc<int>(nnzL);
  C->mapL = C->alloc<int>(nnzL);
  C->Ltrp = C->alloc<int>(n + 1);
  C->Ltci = C->alloc<int>(nnzL);
  C->mapLt = C->alloc<int>(nnzL);
  C->levL = C->alloc<int>(n);
  C->levLt = C->alloc<int>(n);
  C->Lv = C->alloc<double>(nnzL);
  C->Ltv = C->alloc<double>(nnzL);
  C->Lv32 = C->alloc<float>(nnzL);
  C->Ltv32 = C->alloc<float>(nnzL);
  HIPCHK(hipMemcpyAsync(C->Lrp, a.Lrp.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice, C->st));
  HIPCHK(hipMemcpyAsync(C->Lci, a.Lci.data(), sizeof(int) * nnzL, hipMemcpyHostToDevice, C->st));
  HIPCHK(hipMemcpyAsync(C->mapL, a.mapL.data(), sizeof(int) * nnzL, hipMemcpyHostToDevice, C->st));
  HIPCHK(hipMemcpyAsync(C->Ltrp, a.Ltrp.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice, C->st));
  HIPCHK(hipMemcpyAsync(C->Ltci, a.Ltci.data(), sizeof(int) * nnzL, hipMemcpyHostToDevice, C->st));
  HIPCHK(hipMemcpyAsync(C->mapLt, a.mapLt.data(), sizeof(int) * nnzL, hipMemcpyHostToDevice, C->st));
  HIPCHK(hipMemcpyAsync(C->levL, a.levL.rows.data(), sizeof(int) * n, hipMemcpyHostToDevice, C->st));
  HIPCHK(hipMemcpyAsync(C->levLt, a.levLt.rows.data(), sizeof(int) * n, hipMemcpyHostToDevice, C->st));
  // Long rows (more than nr dependencies) through chains of virtual partial-sum rows, so
  // every row of the block solve takes its branch-free path
  bool split = true;
  if (const char *e = getenv("BNX_SPLIT_LONG")) split = atoi(e) != 0;  // tuning override
  // Level-pair substitution (compress_both) when it shortens both dependency chains below
  // 3/4 and keeps every row within kNRC dependencies, or, with split schedules, grows the
  // entries by at most half: the fp32 solves then run the two compressed systems, whose
  // values finish_factor derives from the factor's.  It is tried only when a level holds
  // fewer than kLpsRowsPerLevel rows on average: thin levels cost their hand-over latency
  // and halving them pays (500k-node geometric graph, 176 rows per level: fp32 solve 460
  // against 545 us), while a compressed level of a wide one carries twice the rows and up
  // to six dependencies per row, costs about twice as much, and the right-hand-side
  // transform adds gathers to every solve (100^3 grid, 3356 rows per level: 108 against
  // 103 us in the eigensolve, 3.26 against 3.47 eigenpairs/s mixed).
  bool lps = (double)n / std::max(1, a.levL.nlev) < kLpsRowsPerLevel;
  if (const char *e = getenv("BNX_LPS")) lps = atoi(e) != 0;  // override: 1 try it, 0 never
  SolveSys Sf, Sb;  // host copies, kept for the rank-order transforms of the block schedules
  {
    C->lps = lps && compress_both(a, split, Sf, Sb);
    if (C->lps) {
      Analysis &S = C->anS;
      S = Analysis{};
      S.n = n;
      S.Lrp = Sf.rp;
      S.Lci = Sf.ci;
      S.Ltrp = Sb.rp;
      S.Ltci = Sb.ci;
      S.nnzL = Sf.nnz;
      levels_from(n, Sf.level, S.levL);
      levels_from(n, Sb.level, S.levLt);
      auto up = [&](const std::vector<int> &v) {
        int *d = C->alloc<int>(std::max<size_t>(v.size(), 1));
        if (!v.empty()) HIPCHK(hipMemcpyAsync(d, v.data(), sizeof(int) * v.size(), hipMemcpyHostToDevice, C->st));
        return d;
      };
      for (int d = 0; d < 2; d++) {
        const SolveSys &Q = d == 0 ? Sf : Sb;
        auto &D = C->sys[d];
        D.nnz = Q.nnz;
        D.nm = (int)Q.mj.size();
        D.rp = up(Q.rp);
        D.ci = up(Q.ci);
        D.lev = up(d == 0 ? S.levL.rows : S.levLt.rows);
        D.direct = up(Q.direct);
        D.tp = up(Q.tp);
        D.ta = up(Q.ta);
        D.tb = up(Q.tb);
        D.tc = up(Q.tc);
        D.mp = up(Q.mp);
        D.mj = up(Q.mj);
        D.ma = up(Q.ma);
        D.mc = up(Q.mc);
        D.v = C->alloc<double>(Q.nnz);
        D.v32 = C->alloc<float>(Q.nnz);
        D.mv = C->alloc<double>(std::max(D.nm, 1));
        D.mv32 = C->alloc<float>(std::max(D.nm, 1));
      }
      C->sync();  // host vectors go out of scope
    }
  }
  for (int pr = 0; pr < 2; pr++) {
    std::vector<int> prow, pstart;
    // Block size target: larger blocks cross fewer block boundaries, smaller ones
    // keep more waves per level busy; measured best near 7k (FP64) and 12k (FP32)
    // rows on the 7-point 100^3 grid, and 8k in FP32 for the level-compressed systems
    // (their levels hold twice the rows: 256 blocks beat 128).
    const bool cmp = C->lps && pr == 1;  // FP32 schedules of the compressed systems
    const Analysis &sa = cmp ? C->anS : a;
    int nr = slots_for(sa, cmp);
    // rows of many dependencies (27-point elasticity blocks, ~38 per row): six slots shorten
    // their chains of virtual rows (measured 7-11 % faster fp64 solves, 3 % fp32); with few (the
    // geometric graph, ~5) the wider rows leave too few blocks and lose
    if (split && !cmp && nr == kNR && (double)(sa.nnzL - sa.n) > 2.0 * kNRC * sa.n) nr = kNRC;
    if (const char *e = getenv("BNX_NR"))  // tuning override: slots of the uncompressed split schedules
      if (split && !cmp && nr > 3 && (atoi(e) == kNR || atoi(e) == kNRC || (atoi(e) == kNRW && pr == 1)))
        nr = atoi(e);
    int cap = pr == 0 ? kBlkTarget64 : (cmp ? kBlkTarget32C : kBlkTarget32);
    if (const char *e = getenv(pr == 0 ? "BNX_BLK_CAP64" : "BNX_BLK_CAP32"))  // tuning override
      cap = atoi(e);
    // the block's right-hand side takes as many LDS values as its ranks: half the LDS for the rest
    const int lds = pr == 0 ? kLdsCap64 : kLdsCap32;
    cap = std::max(256, std::min(cap, lds / 2 - 128));  // 128: padding of a block to whole slices
    if (!partition_rows(sa, cap, prow, pstart, split, nr, cmp ? &a : nullptr)) continue;  // no block schedule
    for (int dir = 0; dir < 2; dir++) {
      BlockSched bs;
      block_schedule(sa, dir == 0, prow, pstart, bs, split, nr);
      int need = 0;  // rows + imports + zero slot + right-hand side of the rows + a dump slot
      for (int q = 0; q < bs.nblocks; q++)
        need = std::max(need, 2 * bs.brows[q] + (bs.iptr[q + 1] - bs.iptr[q]) + 2);
      if (bs.max_lds > lds || need > lds) throw ApiError{BNX_E_STATE, "block schedule exceeds LDS"};
      auto &b = C->blk[dir][pr];
      b.n = bs.n;
      b.nr = bs.nr;
      b.npad = bs.npad;
      b.nblocks = bs.nblocks;
      b.ell = bs.ell;
      b.nexp = bs.nexp;
      auto up = [&](const std::vector<int> &v) {
        int *d = C->alloc<int>(std::max<size_t>(v.size(), 1));
        if (!v.empty())
          HIPCHK(hipMemcpyAsync(d, v.data(), sizeof(int) * v.size(), hipMemcpyHostToDevice, C->st));
        return d;
      };
      b.bptr = up(bs.bptr);
      b.brows = up(bs.brows);
      b.iptr = up(bs.iptr);
      b.isrc = up(bs.isrc);
      b.eptr = up(bs.eptr);
      b.erank = up(bs.erank);
      b.orow = up(bs.orow);
      b.oslot = up(bs.oslot);
      b.perm = up(bs.perm);
      b.slice_ptr = up(bs.slice_ptr);
      b.slice_nnz = up(bs.slice_nnz);
      b.ref = up(bs.ref);
      b.valmap = up(bs.valmap);
      b.diagmap = up(bs.diagmap);
      b.cnt = up(bs.cnt);
      b.ref4 = up(bs.ref4);
      b.valmap4 = up(bs.valmap4);
      if (cmp) {  // the compressed system's right-hand-side transform, in rank order
        const SolveSys &Q = dir == 0 ? Sf : Sb;
        int mw = 0;
        for (int i = 0; i < n; i++) mw = std::max(mw, Q.mp[i + 1] - Q.mp[i]);
        std::vector<int> mjr((size_t)mw * bs.npad, -1), mtr((size_t)mw * bs.npad, 0);
        for (int k = 0; k < bs.npad; k++) {
          const int i = bs.perm[k];
          if (i < 0) continue;
          for (int t = Q.mp[i]; t < Q.mp[i + 1]; t++) {
            mjr[(size_t)(t - Q.mp[i]) * bs.npad + k] = Q.mj[t];
            mtr[(size_t)(t - Q.mp[i]) * bs.npad + k] = t;
          }
        }
        b.mw = mw;
        b.mjr = up(mjr);
        b.mtr = up(mtr);
      }
      const size_t np = (size_t)bs.npad;
      if (pr == 0) {
        b.diag64 = C->alloc<double>(np);
        b.val64 = C->alloc<double>(std::max(bs.ell, 1));
        b.val4_64 = C->alloc<double>((size_t)bs.nr * np);
      } else {
        b.diag32 = C->alloc<float>(np);
        b.val32 = C->alloc<float>(std::max(bs.ell, 1));
        b.val4_32 = C->alloc<float>((size_t)bs.nr * np);
      }
      C->sync();  // host vectors go out of scope
    }
  }
  {
    C->blk_nexp64 = std::max({1, C->blk[0][0].nexp, C->blk[1][0].nexp});
    C->blk_nexp32 = std::max({1, C->blk[0][1].nexp, C->blk[1][1].nexp});
    C->blk_exp64 = C->alloc<double>(2 * (size_t)C->blk_nexp64);
    C->blk_exp32 = C->alloc<float>(2 * (size_t)C->blk_nexp32);
    C->blk_cnt = C->alloc<int>(4);
    launch_blk_reset<double>(C->st, C->blk_exp64, C->blk_nexp64, C->blk_cnt);
    launch_blk_reset<float>(C->st, C->blk_exp32, C->blk_nexp32, C->blk_cnt + 2);
    C->blk_seq[0] = C->blk_seq[1] = 0;
  }
  C->sync();
  C->ta = &a;
}

void finish_factor(bnx_ctx *C);

void factor_impl(bnx_ctx *C, const bnx_factor_opts &o) {
  const double t0 = now_s();
  C->factored = false;  // a failed factorisation leaves no factor behind
  C->solved = false;
  const double shift0 = o.shift0, shift_max = o.shift_max;
  const int n = C->n;
  if (o.ict) {
    // IC(lfil, tau_IC) on the host (ict.hip), then the device structures of its pattern
    std::vector<double> hv(C->nnz);
    HIPCHK(hipMemcpyAsync(hv.data(), C->val, sizeof(double) * C->nnz, hipMemcpyDeviceToHost, C->st));
    C->sync();
    IctFactor F;
    double a = 0.0;
    while (!ict_factor(n, C->an.rp.data(), C->an.ci.data(), hv.data(), o.lfil, o.tau_ic, a, F)) {
      a = (a == 0.0) ? shift0 : 2.0 * a;
      if (shift0 <= 0.0 || a > shift_max) throw ApiError{BNX_E_NOT_SPD, "IC(lfil, tau) breakdown beyond shift_max"};
    }
    // the installed structures serve again when the pattern is the one they were built for
    // (a refactor of the same values, or of values that drop the same entries)
    if (C->ta != &C->anT || C->anT.Lrp != F.rp || C->anT.Lci != F.ci) {
      pattern_of_factor(n, F, C->anT);
      analyse(C->anT);
      if (C->anT.Lci != F.ci) throw ApiError{BNX_E_STATE, "factor pattern mismatch"};
      build_tri(C, C->anT);
    }
    HIPCHK(hipMemcpyAsync(C->Lv, F.v.data(), sizeof(double) * F.v.size(), hipMemcpyHostToDevice, C->st));
    C->shift_used = a;
    finish_factor(C);
    C->sync();  // F goes out of scope
    C->t_factor = now_s() - t0;
    return;
  }
  if (C->ta != &C->an) build_tri(C, C->an);
  const Analysis &an = C->an;
  const int nnzL = an.nnzL;
  double a = 0.0;
  for (;;) {
    hipLaunchKernelGGL(k_ic0_gather, dim3(gridn(nnzL)), dim3(kBlock), 0, C->st, nnzL, C->mapL, C->val, C->Lv);
    HIPCHK(hipMemsetAsync(C->dflag, 0, sizeof(int), C->st));
    for (int l = 0; l < an.levL.nlev; l++) {
      const int r0 = an.levL.ptr[l], r1 = an.levL.ptr[l + 1];
      hipLaunchKernelGGL(k_ic0_level, dim3((r1 - r0 + 127) / 128), dim3(128), 0, C->st, r0, r1, C->levL, C->Lrp,
                         C->Lci, C->Lv, a, C->dflag);
    }
    HIPCHK(hipMemcpyAsync(C->hflag, C->dflag, sizeof(int), hipMemcpyDeviceToHost, C->st));
    C->sync();
    if (C->hflag[0] == 0) break;
    a = (a == 0.0) ? shift0 : 2.0 * a;
    if (shift0 <= 0.0 || a > shift_max) throw ApiError{BNX_E_NOT_SPD, "IC(0) breakdown beyond shift_max"};
  }
  C->shift_used = a;
  finish_factor(C);
  C->t_factor = now_s() - t0;
}

// L^T values, the FP32 copies and the block-schedule value arrays from L (C->Lv).
void finish_factor(bnx_ctx *C) {
  const int nnzL = C->ta->nnzL;
  hipLaunchKernelGGL(k_gather_d, dim3(gridn(nnzL)), dim3(kBlock), 0, C->st, nnzL, C->mapLt, C->Lv, C->Ltv);
  launch_cast<double, float>(C->st, nnzL, C->Lv, C->Lv32);
  launch_cast<double, float>(C->st, nnzL, C->Ltv, C->Ltv32);
  if (C->lps)
    for (int d = 0; d < 2; d++) {
      auto &S = C->sys[d];
      const double *v = d == 0 ? C->Lv : C->Ltv;
      hipLaunchKernelGGL(k_sys_values, dim3(gridn(S.nnz)), dim3(kBlock), 0, C->st, S.nnz, S.direct, S.tp, S.ta, S.tb,
                         S.tc, v, S.v);
      launch_cast<double, float>(C->st, S.nnz, S.v, S.v32);
      if (S.nm > 0) {
        hipLaunchKernelGGL(k_sys_m, dim3(gridn(S.nm)), dim3(kBlock), 0, C->st, S.nm, S.ma, S.mc, v, S.mv);
        launch_cast<double, float>(C->st, S.nm, S.mv, S.mv32);
      }
    }
  for (int dir = 0; dir < 2; dir++) {
    for (int pr = 0; pr < 2; pr++) {
      const double *src = (C->lps && pr == 1) ? C->sys[dir].v : (dir == 0 ? C->Lv : C->Ltv);
      auto &b = C->blk[dir][pr];
      if (b.nblocks == 0) continue;
      const int np = b.npad;
      if (pr == 0) {
        hipLaunchKernelGGL((k_gather_rdiag<double>), dim3(gridn(np)), dim3(kBlock), 0, C->st, np, b.diagmap, src,
                           b.diag64);
        hipLaunchKernelGGL((k_gather_blk<double>), dim3(gridn(b.ell)), dim3(kBlock), 0, C->st, b.ell, b.valmap, src,
                           b.val64);
        hipLaunchKernelGGL((k_gather_blk<double>), dim3(gridn(b.nr * np)), dim3(kBlock), 0, C->st, b.nr * np,
                           b.valmap4, src, b.val4_64);
      } else {
        hipLaunchKernelGGL((k_gather_rdiag<float>), dim3(gridn(np)), dim3(kBlock), 0, C->st, np, b.diagmap, src,
                           b.diag32);
        hipLaunchKernelGGL((k_gather_blk<float>), dim3(gridn(b.ell)), dim3(kBlock), 0, C->st, b.ell, b.valmap, src,
                           b.val32);
        hipLaunchKernelGGL((k_gather_blk<float>), dim3(gridn(b.nr * np)), dim3(kBlock), 0, C->st, b.nr * np,
                           b.valmap4, src, b.val4_32);
      }
    }
  }
  C->sync();
  C->factored = true;
  C->solved = false;
}

template <typename F>
bnx_status guarded(bnx_ctx *C, F &&f) {
  try {
    C->err.clear();
    return f();
  } catch (const ApiError &e) {
    C->err = e.msg;
    return e.code;
  } catch (const HipError &e) {
    C->err = e.msg;
    return BNX_E_HIP;
  } catch (const std::bad_alloc &) {
    C->err = "host allocation failed";
    return BNX_E_NOMEM;
  }
}

void upload_values(bnx_ctx *C, const double *val) {
  HIPCHK(hipMemcpyAsync(C->val, val, sizeof(double) * C->nnz,
                        C->device_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, C->st));
  launch_cast<double, float>(C->st, C->nnz, C->val, C->val32);
  if (C->ell_ptr) {
    hipLaunchKernelGGL((k_gather_blk<double>), dim3(gridn(C->ell_size)), dim3(kBlock), 0, C->st, C->ell_size,
                       C->ell_map, C->val, C->ell_v64);
    hipLaunchKernelGGL((k_gather_blk<float>), dim3(gridn(C->ell_size)), dim3(kBlock), 0, C->st, C->ell_size,
                       C->ell_map, C->val, C->ell_v32);
  }
  // diagonal must be positive
  std::vector<double> hv(C->nnz);
  HIPCHK(hipMemcpyAsync(hv.data(), C->val, sizeof(double) * C->nnz, hipMemcpyDeviceToHost, C->st));
  C->sync();
  for (int i = 0; i < C->n; i++)
    for (int e = C->an.rp[i]; e < C->an.rp[i + 1]; e++)
      if (C->an.ci[e] == i && !(hv[e] > 0.0)) throw ApiError{BNX_E_NOT_SPD, "non-positive diagonal entry"};
  C->factored = false;
  C->solved = false;
}

bool prec_ok(int p) { return p == BNX_FP64 || p == BNX_MIXED; }

}  // namespace

// ================================================================== no-allocation scratch
// Scratch of bnx_ic_apply_noalloc: the temporaries that bnx_ic_apply allocates per call (one n-vector
// of doubles, or three n-vectors of floats), for n <= kNoAllocMaxN.  Each device holds its own copy
// for the life of the process.  Host code never uses the array's name as an address: the device
// address of each device's copy is taken once, with hipGetSymbolAddress, when the first context is
// created on that device, and kept per device.
constexpr int kNoAllocMaxN = 1 << 20;
static __device__ __align__(256) double scratch[(size_t)kNoAllocMaxN * 3 / 2];  // 12 MiB

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxDevices] = {};

// the current device's scratch address (the device of the context being created)
void *scratch_address() {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw ApiError{BNX_E_ARG, "device ordinal out of range for the scratch table"};
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) throw HipError{std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
    g_scratch_addr[dev] = p;
  }
  return g_scratch_addr[dev];
}
}  // namespace

// ================================================================== C-ABI
namespace {
template <typename T>
static void ic_apply_t(bnx_ctx *C, int which, const T *b, T *x, T *tmp, bool events = true) {
  Launch L = C->launch();
  if (!events) L.prof = nullptr;  // the event timing creates events; the no-allocation path records none
  launch_fill<int>(C->st, 1, &C->ctl->err, 0);
  if (which == 0) launch_trsv<T>(L, C->tri<T>(true), b, x, 0, VList<T>{}, nullptr, nullptr);
  else if (which == 1) launch_trsv<T>(L, C->tri<T>(false), b, x, 0, VList<T>{}, nullptr, nullptr);
  else {
    launch_trsv<T>(L, C->tri<T>(true), b, tmp, 0, VList<T>{}, nullptr, nullptr);
    launch_trsv<T>(L, C->tri<T>(false), tmp, x, 0, VList<T>{}, nullptr, nullptr);
  }
  if (C->readctl().err) throw ApiError{BNX_E_BREAKDOWN, "triangular solve wait bound exceeded"};
}

template <typename T>
static void prec_apply_t(bnx_ctx *C, int k, const double *S, const double *R, int m, const double *Q, const double *g,
                         double *out) {
  const int n = C->n;
  const Launch L = C->launch();
  DevCtl *c = C->ctl;
  const bool fp64 = std::is_same<T, double>::value;
  Work<T> w;
  make_work<T>(C, w, k, m);
  std::vector<T *> extra;
  VList<T> SL{}, RL{}, QL{};
  for (int s = 0; s < k; s++) {
    launch_cast<double, T>(C->st, n, S + (size_t)s * n, w.S[s]);
    launch_cast<double, T>(C->st, n, R + (size_t)s * n, w.R[s]);
    SL.p[s] = w.S[s];
    RL.p[s] = w.R[s];
  }
  for (int q = 0; q < m; q++) {
    launch_cast<double, T>(C->st, n, Q + (size_t)q * n, w.Qm + (size_t)q * n);
    QL.p[q] = w.Qm + (size_t)q * n;
  }
  launch_cast<double, T>(C->st, n, g, w.g);
  HIPCHK(hipMemsetAsync(&c->err, 0, sizeof(int), C->st));
  gram_full<T>(C, k, SL, RL, m, QL);
  VList<T> X{}, Y{};
  for (int s = 0; s < k; s++) {
    X.p[s] = SL.p[s];
    Y.p[s] = w.g;
  }
  for (int q = 0; q < m; q++) {
    X.p[k + q] = QL.p[q];
    Y.p[k + q] = w.g;
  }
  int nb = launch_multidot<T, T>(L, n, k + m, X, Y, area(L, 3), nullptr);
  if (k + m == 0) nb = 1;
  hipLaunchKernelGGL(c_prec_a, dim3(1), dim3(kBlock), 0, C->st, c, area(L, 3), nb, k, m);
  launch_trsv<T>(L, C->tri<T>(true), w.g, w.z, k, RL, c->a, nullptr);
  launch_trsv<T>(L, C->tri<T>(false), w.z, w.c0, 0, RL, nullptr, nullptr);
  VList<T> mX{}, mY{};
  for (int s = 0; s < k; s++) {
    mX.p[s] = RL.p[s];
    mY.p[s] = w.c0;
  }
  for (int q = 0; q < m; q++) {
    mX.p[k + q] = QL.p[q];
    mY.p[k + q] = w.c0;
  }
  mX.p[k + m] = w.g;
  mY.p[k + m] = w.c0;
  nb = launch_multidot<T, T>(L, n, k + m + 1, mX, mY, area(L, 3), nullptr);
  hipLaunchKernelGGL(c_pcg_beta, dim3(1), dim3(kBlock), 0, C->st, c, area(L, 3), nb);
  hipLaunchKernelGGL((k_pcg_newp<T, 0>), dim3(gridn(n)), dim3(kBlock), 0, C->st, n, c, w.c0, k, SL, m, QL, w.p, 0, 0,
                     VList<T>{}, nullptr);
  launch_cast<T, double>(C->st, n, w.p, out);
  DevCtl h = C->readctl();
  free_work<T>(C, w);
  if (h.err) throw ApiError{BNX_E_BREAKDOWN, "triangular solve wait bound exceeded"};
  (void)fp64;
}

template <typename T>
static void corr_solve_t(bnx_ctx *C, int m, const double *Q, int k, const double *S, const double *R, double tol_pcg,
                         int itmax_pcg, double tau, int exit_rule, double xi, double *s, int *its, int *reason) {
  const int n = C->n;
  Work<T> w;
  make_work<T>(C, w, k, m);
  double *u = C->alloc<double>(n), *Au = C->alloc<double>(n), *r = C->alloc<double>(n);
  HIPCHK(hipMemcpyAsync(u, Q + (size_t)(m - 1) * n, sizeof(double) * n, hipMemcpyDeviceToDevice, C->st));
  HIPCHK(hipMemsetAsync(&C->ctl->err, 0, sizeof(int), C->st));
  outer_eval<T>(C, u, Au, r, w.u, w.Au, w.r);
  const double theta = C->readctl().otheta;
  VList<T> SL{}, RL{}, QL{};
  for (int t = 0; t < k; t++) {
    launch_cast<double, T>(C->st, n, S + (size_t)t * n, w.S[t]);
    launch_cast<double, T>(C->st, n, R + (size_t)t * n, w.R[t]);
    SL.p[t] = w.S[t];
    RL.p[t] = w.R[t];
  }
  for (int q = 0; q < m; q++) {
    launch_cast<double, T>(C->st, n, Q + (size_t)q * n, w.Qm + (size_t)q * n);
    QL.p[q] = w.Qm + (size_t)q * n;
  }
  gram_full<T>(C, k, SL, RL, m, QL);
  VList<T> AQ{};
  for (int q = 0; q < m; q++) {
    launch_spmv<T>(C->launch(), C->mat<T>(), QL.p[q], w.AQm + (size_t)q * n, 0, VList<T>{}, 0, VList<T>{}, nullptr,
                   nullptr);
    AQ.p[q] = w.AQm + (size_t)q * n;
  }
  PcgParams P;
  P.theta = theta;
  P.tol_pcg = tol_pcg;
  P.itmax = itmax_pcg;
  P.tau = tau;
  P.exit_rule = exit_rule;
  P.xi = xi;
  P.sgn = -1.0;
  P.eigtest = 1;
  pcg<T>(C, w, P, w.r, m, QL, AQ, k, SL, RL, w.u, w.Au, w.s, its, reason);
  launch_cast<T, double>(C->st, n, w.s, s);
  C->sync();
  C->release(u);
  C->release(Au);
  C->release(r);
  free_work<T>(C, w);
}

template <typename T>
static void dacg_t(bnx_ctx *C, int m, const double *Qt, const double *x0, double tol, int itmax, double *x, int *its) {
  const int n = C->n;
  Work<T> w;
  make_work<T>(C, w, 0, m);
  double *x64 = C->alloc<double>(n), *tmp = C->alloc<double>(n);
  VList<double> Q64{};
  VList<T> QT{};
  for (int q = 0; q < m; q++) {
    Q64.p[q] = Qt + (size_t)q * n;
    launch_cast<double, T>(C->st, n, Qt + (size_t)q * n, w.Qm + (size_t)q * n);
    QT.p[q] = w.Qm + (size_t)q * n;
  }
  HIPCHK(hipMemcpyAsync(x64, x0, sizeof(double) * n, hipMemcpyDeviceToDevice, C->st));
  HIPCHK(hipMemsetAsync(&C->ctl->err, 0, sizeof(int), C->st));
  cgs2_normalize(C, x64, tmp, m, Q64);
  launch_cast<double, T>(C->st, n, x64, w.x);
  long long mvp = 0;
  *its = dacg<T>(C, w, m, QT, tol, itmax, &mvp);
  launch_cast<T, double>(C->st, n, w.x, x);
  C->sync();
  C->release(x64);
  C->release(tmp);
  free_work<T>(C, w);
}

}  // namespace

extern "C" {

void bnx_default_solve_opts(bnx_solve_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->p = 10;
  o->tol = 1e-8;
  o->itmax = 100;
  o->tol_dacg = 1e-2;
  o->itmax_dacg = 5000;
  o->tol_pcg = 1e-2;
  o->itmax_pcg = 20;
  o->kmax = 5;
  o->precision = BNX_FP64;
  o->exit_rule = 1;
  o->exit_xi = 0.1;
  o->seed = 0;
  o->x0 = nullptr;
  o->keep_bfgs = 0;
  o->newton = 1;
  o->bfgs_full = 0;
  o->jd = 0;
  o->jd_mmin = 5;
  o->jd_mmax = 10;
}

void bnx_default_factor_opts(bnx_factor_opts *o) {
  if (!o) return;
  o->shift0 = 1e-3;
  o->shift_max = 1.0;
  o->ict = 0;
  o->lfil = 30;
  o->tau_ic = 1e-2;
}

bnx_status bnx_create_csr(bnx_ctx **out, int64_t n, int64_t nnz, const int32_t *rowptr, const int32_t *col,
                          const double *val, int device_ptrs, void *hip_stream) {
  if (!out) return BNX_E_ARG;
  *out = nullptr;
  if (n < 1 || nnz < n || n > INT32_MAX || nnz > INT32_MAX || !rowptr || !col || !val) return BNX_E_ARG;
  bnx_ctx *C = new (std::nothrow) bnx_ctx;
  if (!C) return BNX_E_NOMEM;
  C->n = (int)n;
  C->nnz = (int)nnz;
  C->device_ptrs = device_ptrs ? 1 : 0;
  C->st = (hipStream_t)hip_stream;
  bnx_status s = guarded(C, [&]() -> bnx_status {
    C->scratch = scratch_address();
    C->an.n = C->n;
    C->an.nnz = C->nnz;
    C->an.rp.resize(n + 1);
    C->an.ci.resize(nnz);
    if (device_ptrs) {
      HIPCHK(hipMemcpy(C->an.rp.data(), rowptr, sizeof(int) * (n + 1), hipMemcpyDeviceToHost));
      HIPCHK(hipMemcpy(C->an.ci.data(), col, sizeof(int) * nnz, hipMemcpyDeviceToHost));
    } else {
      std::memcpy(C->an.rp.data(), rowptr, sizeof(int) * (n + 1));
      std::memcpy(C->an.ci.data(), col, sizeof(int) * nnz);
    }
    std::string v = validate_csr(C->n, C->nnz, C->an.rp.data(), C->an.ci.data());
    if (!v.empty()) throw ApiError{BNX_E_ARG, v};
    analyse(C->an);
    C->group = spmv_group((double)nnz / (double)n);
    // SELL-64 copy for the SpMV when its padding stays small: slice s holds rows 64s..64s+63, entry e of
    // lane l at ell_ptr[s] + 64 e + l; padding reads x[row] with weight 0
    {
      const int ns = (n + 63) / 64;
      std::vector<int> eptr(ns + 1, 0), elen(ns, 0);
      for (int sl = 0; sl < ns; sl++) {
        int mx = 0;
        for (int i = sl * 64; i < std::min<int>(n, sl * 64 + 64); i++) mx = std::max(mx, C->an.rp[i + 1] - C->an.rp[i]);
        elen[sl] = mx;
        eptr[sl + 1] = eptr[sl] + 64 * mx;
      }
      const long long esz = eptr[ns];
      if (esz <= 5LL * nnz / 4 && esz < INT32_MAX && !getenv("BNX_NO_ELL")) {
        std::vector<int> ecol(esz), emap(esz, -1);
        for (int sl = 0; sl < ns; sl++)
          for (int l = 0; l < 64; l++) {
            const int i = sl * 64 + l;
            for (int e = 0; e < elen[sl]; e++) {
              const size_t at = (size_t)eptr[sl] + 64 * e + l;
              const int q = i < n ? C->an.rp[i] + e : -1;
              if (i < n && q < C->an.rp[i + 1]) {
                ecol[at] = C->an.ci[q];
                emap[at] = q;
              } else {
                ecol[at] = i < n ? i : 0;
              }
            }
          }
        C->ell_size = (int)esz;
        C->ell_ptr = C->alloc<int>(ns + 1);
        C->ell_len = C->alloc<int>(ns);
        C->ell_col = C->alloc<int>(esz);
        C->ell_map = C->alloc<int>(esz);
        C->ell_v64 = C->alloc<double>(esz);
        C->ell_v32 = C->alloc<float>(esz);
        HIPCHK(hipMemcpyAsync(C->ell_ptr, eptr.data(), sizeof(int) * (ns + 1), hipMemcpyHostToDevice, C->st));
        HIPCHK(hipMemcpyAsync(C->ell_len, elen.data(), sizeof(int) * ns, hipMemcpyHostToDevice, C->st));
        HIPCHK(hipMemcpyAsync(C->ell_col, ecol.data(), sizeof(int) * esz, hipMemcpyHostToDevice, C->st));
        HIPCHK(hipMemcpyAsync(C->ell_map, emap.data(), sizeof(int) * esz, hipMemcpyHostToDevice, C->st));
        C->sync();  // host vectors go out of scope
      }
    }
    build_tri(C, C->an);
    if (const char *e = getenv("BNX_SF_WAVES")) C->sf_waves = atoi(e);  // tuning override of the solve window
    C->rp = C->alloc<int>(n + 1);
    C->ci = C->alloc<int>(nnz);
    C->val = C->alloc<double>(nnz);
    C->val32 = C->alloc<float>(nnz);
    C->ctl = C->alloc<DevCtl>(1);
    C->part = C->alloc<double>((size_t)kAreas * kPartSlots * kNBMax);
    C->counter = C->alloc<int>(4);
    HIPCHK(hipMemsetAsync(C->counter, 0, 4 * sizeof(int), C->st));
    C->dflag = C->alloc<int>(4);
    HIPCHK(hipHostMalloc((void **)&C->hctl, sizeof(DevCtl), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void **)&C->hflag, 4 * sizeof(int), hipHostMallocMapped));
    HIPCHK(hipHostGetDevicePointer((void **)&C->dhflag, C->hflag, 0));
    HIPCHK(hipMemsetAsync(C->ctl, 0, sizeof(DevCtl), C->st));
    HIPCHK(hipMemcpyAsync(C->rp, C->an.rp.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice, C->st));
    HIPCHK(hipMemcpyAsync(C->ci, C->an.ci.data(), sizeof(int) * nnz, hipMemcpyHostToDevice, C->st));
    upload_values(C, val);
    return BNX_OK;
  });
  if (s != BNX_OK) {
    fprintf(stderr, "bnx_create_csr: %s\n", C->err.c_str());
    delete C;
    return s;
  }
  *out = C;
  return BNX_OK;
}

bnx_status bnx_set_values(bnx_ctx *C, const double *val) {
  if (!C || !val) return BNX_E_ARG;
  return guarded(C, [&]() -> bnx_status {
    upload_values(C, val);
    return BNX_OK;
  });
}

bnx_status bnx_factor(bnx_ctx *C, const bnx_factor_opts *opts) {
  if (!C) return BNX_E_ARG;
  bnx_factor_opts o;
  bnx_default_factor_opts(&o);
  if (opts) o = *opts;
  if (o.ict && (o.lfil < 0 || !(o.tau_ic >= 0.0))) return BNX_E_ARG;
  return guarded(C, [&]() -> bnx_status {
    factor_impl(C, o);
    return BNX_OK;
  });
}

bnx_status bnx_factor_info(const bnx_ctx *C, long long *nnz_L, double *fill, int *levels_L, int *levels_Lt,
                           double *shift_used) {
  if (!C) return BNX_E_ARG;
  if (!C->factored || !C->ta) return BNX_E_STATE;
  if (nnz_L) *nnz_L = C->ta->nnzL;
  if (fill) *fill = (double)C->ta->nnzL / (double)C->an.nnzL;
  if (levels_L) *levels_L = C->ta->levL.nlev;
  if (levels_Lt) *levels_Lt = C->ta->levLt.nlev;
  if (shift_used) *shift_used = C->shift_used;
  return BNX_OK;
}

bnx_status bnx_solve(bnx_ctx *C, const bnx_solve_opts *opts, double *evals, double *evecs, bnx_stats *stats) {
  if (!C || !opts || !evals) return BNX_E_ARG;
  return guarded(C, [&]() -> bnx_status {
    const bnx_solve_opts &o = *opts;
    if (!C->factored) throw ApiError{BNX_E_STATE, "bnx_factor must precede bnx_solve"};
    if (o.p < 1 || o.p > BNX_MAX_P || o.p > C->n) throw ApiError{BNX_E_ARG, "p out of range"};
    if (o.kmax < 0 || o.kmax > BNX_MAX_KMAX) throw ApiError{BNX_E_ARG, "kmax out of range"};
    if (!prec_ok(o.precision)) throw ApiError{BNX_E_ARG, "unknown precision"};
    if (o.itmax < 0 || o.itmax_pcg < 1 || o.itmax_dacg < 0 || !(o.tol > 0)) throw ApiError{BNX_E_ARG, "bad iteration parameters"};
    if (o.jd && (o.jd_mmin < 1 || o.jd_mmax <= o.jd_mmin || o.jd_mmax > kJdMax))
      throw ApiError{BNX_E_ARG, "Jacobi-Davidson needs 1 <= jd_mmin < jd_mmax <= 16"};
    if (o.precision == BNX_FP64) return solve_impl<double>(C, o, evals, evecs, stats);
    return solve_impl<float>(C, o, evals, evecs, stats);
  });
}

bnx_status bnx_set_adjoint_params(bnx_ctx *C, double tol_adj, int itmax_adj) {
  if (!C || !(tol_adj > 0) || itmax_adj < 1) return BNX_E_ARG;
  C->adj_tol = tol_adj;
  C->adj_itmax = itmax_adj;
  return BNX_OK;
}

bnx_status bnx_backward(bnx_ctx *C, const double *g_evals, const double *g_evecs, double *g_vals) {
  if (!C || !g_evals || !g_vals) return BNX_E_ARG;
  return guarded(C, [&]() -> bnx_status {
    if (!C->solved) throw ApiError{BNX_E_STATE, "bnx_backward needs a preceding bnx_solve"};
    const int n = C->n, p = C->p_last;
    double *gv = g_vals, *GV = (double *)g_evecs;
    std::vector<double *> tmp;
    if (!C->device_ptrs) {
      gv = C->alloc<double>(C->nnz);
      tmp.push_back(gv);
      if (g_evecs) {
        GV = C->alloc<double>((size_t)n * p);
        tmp.push_back(GV);
        HIPCHK(hipMemcpyAsync(GV, g_evecs, sizeof(double) * n * p, hipMemcpyHostToDevice, C->st));
      }
    }
    struct G {
      bnx_ctx *C;
      std::vector<double *> &t;
      ~G() {
        for (double *q : t) C->release(q);
      }
    } g{C, tmp};
    const std::string missed = C->prec_last == BNX_FP64 ? backward_impl<double>(C, g_evals, GV, gv)
                                                         : backward_impl<float>(C, g_evals, GV, gv);
    if (!C->device_ptrs) {
      HIPCHK(hipMemcpyAsync(g_vals, gv, sizeof(double) * C->nnz, hipMemcpyDeviceToHost, C->st));
      C->sync();
    }
    if (!missed.empty()) {
      C->err = missed;
      return BNX_NOT_CONVERGED;
    }
    return BNX_OK;
  });
}

const char *bnx_last_error(const bnx_ctx *C) { return C ? C->err.c_str() : "null context"; }

void bnx_destroy(bnx_ctx *C) {
  if (!C) return;
  (void)hipStreamSynchronize(C->st);
  delete C;
}

bnx_status bnx_set_profiling(bnx_ctx *C, int on) {
  if (!C) return BNX_E_ARG;
  return guarded(C, [&]() -> bnx_status {
    C->sync();
    C->prof.reset();
    C->prof.on = on != 0;
    return BNX_OK;
  });
}

bnx_status bnx_kernel_time(bnx_ctx *C, int kernel, double *ms_total, long long *launches) {
  if (!C || kernel < 0 || kernel >= Profiler::kIds || !ms_total || !launches) return BNX_E_ARG;
  return guarded(C, [&]() -> bnx_status {
    C->sync();
    C->prof.drain();
    *ms_total = C->prof.ms[kernel];
    *launches = C->prof.count[kernel];
    return BNX_OK;
  });
}

bnx_status bnx_probe_latency(bnx_ctx *C, int kind, int hops, double *us_per_hop) {
  if (!C || kind < 0 || kind > 1 || hops < 2 || hops > kProbeHopsMax || !us_per_hop) return BNX_E_ARG;
  return guarded(C, [&]() -> bnx_status {
    if (!C->probe_flags) C->probe_flags = C->alloc<int>(kProbeHopsMax);
    HIPCHK(hipMemsetAsync(&C->ctl->err, 0, sizeof(int), C->st));
    hipEvent_t a, b;
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&b));
    launch_probe(C->st, kind, 2, C->probe_flags, C->counter + 1, &C->ctl->err);  // warm-up
    HIPCHK(hipEventRecord(a, C->st));
    launch_probe(C->st, kind, hops, C->probe_flags, C->counter + 1, &C->ctl->err);
    HIPCHK(hipEventRecord(b, C->st));
    HIPCHK(hipGetLastError());
    C->sync();
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (C->readctl().err) throw ApiError{BNX_E_BREAKDOWN, "latency probe wait bound exceeded"};
    *us_per_hop = 1000.0 * ms / hops;
    return BNX_OK;
  });
}

bnx_status bnx_set_trsv_mode(bnx_ctx *C, int mode) {
  if (!C || mode < 0 || mode > 2) return BNX_E_ARG;
  C->trsv_mode = mode;
  return BNX_OK;
}

// ------------------------------------------------------------------ step-level entry points
bnx_status bnx_spmv(bnx_ctx *C, int precision, const double *x, double *y) {
  if (!C || !x || !y || !prec_ok(precision)) return BNX_E_ARG;
  return guarded(C, [&]() -> bnx_status {
    const Launch L = C->launch();
    if (precision == BNX_FP64) {
      launch_spmv<double>(L, C->mat<double>(), x, y, 0, VList<double>{}, 0, VList<double>{}, nullptr, nullptr);
    } else {
      float *xf = C->alloc<float>(C->n), *yf = C->alloc<float>(C->n);
      launch_cast<double, float>(C->st, C->n, x, xf);
      launch_spmv<float>(L, C->mat<float>(), xf, yf, 0, VList<float>{}, 0, VList<float>{}, nullptr, nullptr);
      launch_cast<float, double>(C->st, C->n, yf, y);
      C->sync();
      C->release(xf);
      C->release(yf);
    }
    C->sync();
    return BNX_OK;
  });
}

bnx_status bnx_ic_apply(bnx_ctx *C, int precision, int which, const double *b, double *x) {
  if (!C || !b || !x || !prec_ok(precision) || which < 0 || which > 2) return BNX_E_ARG;
  return guarded(C, [&]() -> bnx_status {
    if (!C->factored) throw ApiError{BNX_E_STATE, "bnx_factor must precede bnx_ic_apply"};
    const int n = C->n;
    if (precision == BNX_FP64) {
      double *tmp = C->alloc<double>(n);
      ic_apply_t<double>(C, which, b, x, tmp);
      C->release(tmp);
    } else {
      float *bf = C->alloc<float>(n), *xf = C->alloc<float>(n), *tf = C->alloc<float>(n);
      launch_cast<double, float>(C->st, n, b, bf);
      ic_apply_t<float>(C, which, bf, xf, tf);
      launch_cast<float, double>(C->st, n, xf, x);
      C->sync();
      C->release(bf);
      C->release(xf);
      C->release(tf);
    }
    return BNX_OK;
  });
}

bnx_status bnx_ic_apply_noalloc(bnx_ctx *C, int precision, int which, const double *b, double *x) {
  if (!C || !b || !x || !prec_ok(precision) || which < 0 || which > 2) return BNX_E_ARG;
  return guarded(C, [&]() -> bnx_status {
    if (!C->factored) throw ApiError{BNX_E_STATE, "bnx_factor must precede bnx_ic_apply_noalloc"};
    const int n = C->n;
    if (n > kNoAllocMaxN)
      throw ApiError{BNX_E_ARG, "bnx_ic_apply_noalloc: n = " + std::to_string(n) + " exceeds its scratch (n <= " +
                                    std::to_string(kNoAllocMaxN) + "); use bnx_ic_apply"};
    if (!C->scratch) throw ApiError{BNX_E_STATE, "no scratch address for this context's device"};
    if (precision == BNX_FP64) {
      ic_apply_t<double>(C, which, b, x, static_cast<double *>(C->scratch), false);
    } else {
      float *bf = static_cast<float *>(C->scratch), *xf = bf + n, *tf = xf + n;
      launch_cast<double, float>(C->st, n, b, bf);
      ic_apply_t<float>(C, which, bf, xf, tf, false);
      launch_cast<float, double>(C->st, n, xf, x);
      C->sync();
    }
    return BNX_OK;
  });
}

bnx_status bnx_prec_apply(bnx_ctx *C, int precision, int k, const double *S, const double *R, int m, const double *Q,
                          const double *g, double *c) {
  if (!C || !g || !c || !prec_ok(precision) || k < 0 || k > BNX_MAX_KMAX || m < 0 || m > BNX_MAX_P + 1)
    return BNX_E_ARG;
  if ((k > 0 && (!S || !R)) || (m > 0 && !Q)) return BNX_E_ARG;
  return guarded(C, [&]() -> bnx_status {
    if (!C->factored) throw ApiError{BNX_E_STATE, "bnx_factor must precede bnx_prec_apply"};
    if (precision == BNX_FP64) prec_apply_t<double>(C, k, S, R, m, Q, g, c);
    else prec_apply_t<float>(C, k, S, R, m, Q, g, c);
    return BNX_OK;
  });
}

bnx_status bnx_correction_solve(bnx_ctx *C, int precision, int m, const double *Q, int k, const double *S,
                                const double *R, double tol_pcg, int itmax_pcg, double tau, int exit_rule,
                                double exit_xi, double *s, int *its, int *reason) {
  if (!C || !Q || !s || !its || !reason || !prec_ok(precision) || m < 1 || m > BNX_MAX_P + 1 || k < 0 ||
      k > BNX_MAX_KMAX || itmax_pcg < 1)
    return BNX_E_ARG;
  if (k > 0 && (!S || !R)) return BNX_E_ARG;
  return guarded(C, [&]() -> bnx_status {
    if (!C->factored) throw ApiError{BNX_E_STATE, "bnx_factor must precede bnx_correction_solve"};
    if (precision == BNX_FP64) corr_solve_t<double>(C, m, Q, k, S, R, tol_pcg, itmax_pcg, tau, exit_rule, exit_xi, s, its, reason);
    else corr_solve_t<float>(C, m, Q, k, S, R, tol_pcg, itmax_pcg, tau, exit_rule, exit_xi, s, its, reason);
    return BNX_OK;
  });
}

bnx_status bnx_dacg(bnx_ctx *C, int precision, int m, const double *Qt, const double *x0, double tol, int itmax,
                    double *x, int *its) {
  if (!C || !x0 || !x || !its || !prec_ok(precision) || m < 0 || m > BNX_MAX_P || itmax < 0 || (m > 0 && !Qt))
    return BNX_E_ARG;
  return guarded(C, [&]() -> bnx_status {
    if (!C->factored) throw ApiError{BNX_E_STATE, "bnx_factor must precede bnx_dacg"};
    if (precision == BNX_FP64) dacg_t<double>(C, m, Qt, x0, tol, itmax, x, its);
    else dacg_t<float>(C, m, Qt, x0, tol, itmax, x, its);
    return BNX_OK;
  });
}

}  // extern "C"
