// Dot reductions of the bnx library: per-block partials summed in a fixed order by one 256-thread block,
// either in a control launch after the producer (reduce_parts) or by the producer's own last block
// (reduce_parts_fused).
#pragma once

#include "internal.h"

namespace bnx {

template <typename T>
__device__ __forceinline__ T wsum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Deterministic reduction of D partial areas (part[d*nb + b], nb <= kNBMax: the areas are sized for that)
// into out[d], in a 256-thread block.  Lane l sums slots l + 64 j into eight sums a[j mod 8] in increasing
// j, then adds the eight in a fixed tree, so the result depends on nb only.  The partials were just
// written by workgroups on every XCD and are read from far memory: a wave issues all of its lanes' loads
// of two dots together (dots d and d + 4).
__device__ __forceinline__ double sum_slots(const double (&v)[kNBMax / 64], int lane, int nb) {
  double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int j = 0; j < kNBMax / 64; j++)
    if (lane + 64 * j < nb) a[j & 7] += v[j];
  return wsum(((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7])));
}

// wfirst: the wave that takes dot 0 (so that two calls can run on different waves); sync: end with a barrier
// (the second of two such calls must).
__device__ inline void reduce_parts(const double *part, int nb, int D, double *out, int wfirst = 0, bool sync = true) {
  constexpr int PL = kNBMax / 64;
  const int lane = threadIdx.x & 63, w = ((threadIdx.x >> 6) - wfirst) & 3;
  for (int d0 = w; d0 < D; d0 += 8) {
    const int d1 = d0 + 4;
    const double *p0 = part + (size_t)d0 * nb, *p1 = part + (size_t)(d1 < D ? d1 : d0) * nb;
    double v0[PL], v1[PL];
#pragma unroll
    for (int j = 0; j < PL; j++) {
      v0[j] = lane + 64 * j < nb ? p0[lane + 64 * j] : 0.0;
      v1[j] = lane + 64 * j < nb && d1 < D ? p1[lane + 64 * j] : 0.0;
    }
    const double s0 = sum_slots(v0, lane, nb);
    const double s1 = sum_slots(v1, lane, nb);
    if (lane == 0) {
      out[d0] = s0;
      if (d1 < D) out[d1] = s1;
    }
  }
  if (sync) __syncthreads();
}

// ---- reductions fused into the producing launch (no control launch after it)
// Each block stores its partials with device-scope stores; the grid's last block waits until every slot
// holds its partial, sums them in the order of reduce_parts (bit-identical to the two-launch form) and
// puts the empty mark back.  Between launches every slot of the fused area holds that mark, a signalling-NaN
// bit pattern that no arithmetic yields (arithmetic on a NaN gives a quiet NaN).  The waiting block is
// one of the grid's own, and every other block of the grid is resident or will be, so the wait ends; the
// bound only turns a broken invariant into an error.  A launch with more than kNBMax blocks is never fused.
constexpr unsigned long long kEmptyMark = 0x7FF4DEAD7FF4DEADull;
constexpr int kFusedArea = kAreas - 1;
constexpr int kFusedSpin = 1 << 22;

// A block's partial of one dot: a plain store, or a device-scope one for a fused reduction.
__device__ __forceinline__ void store_partial(double *slot, double v, bool dev) {
  if (dev)
    __hip_atomic_store((unsigned long long *)slot, (unsigned long long)__double_as_longlong(v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  else
    *slot = v;
}

// Returns false (in every thread) when the wait bound ran out.  Forced inline, like the control steps that
// call it: as a call it would make every producer kernel reserve the callee's registers (280 VGPRs).
__device__ __forceinline__ bool reduce_parts_fused(double *part, int nb, int D, double *out) {
  constexpr int PL = kNBMax / 64;
  __shared__ int bad;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  for (int d = w; d < D; d += 4) {
    unsigned long long *p = (unsigned long long *)(part + (size_t)d * nb);
    unsigned long long v[PL];
#pragma unroll
    for (int j = 0; j < PL; j++)
      v[j] = lane + 64 * j < nb ? __hip_atomic_load(p + lane + 64 * j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                : 0ull;
    for (int left = kFusedSpin;;) {
      bool pend = false;
#pragma unroll
      for (int j = 0; j < PL; j++) pend = pend || (lane + 64 * j < nb && v[j] == kEmptyMark);
      if (__ballot(pend) == 0) break;
      if (--left == 0) {
        if (lane == 0) bad = 1;
        break;
      }
#pragma unroll
      for (int j = 0; j < PL; j++)
        if (lane + 64 * j < nb && v[j] == kEmptyMark)
          v[j] = __hip_atomic_load(p + lane + 64 * j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // the summation of reduce_parts
    double vd[PL];
#pragma unroll
    for (int j = 0; j < PL; j++) vd[j] = __longlong_as_double((long long)v[j]);
    const double s = sum_slots(vd, lane, nb);
    if (lane == 0) out[d] = s;
#pragma unroll
    for (int j = 0; j < PL; j++)
      if (lane + 64 * j < nb) __hip_atomic_store(p + lane + 64 * j, kEmptyMark, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  return bad == 0;
}

}  // namespace bnx
