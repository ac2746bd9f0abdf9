// Cross-lane reductions over a 64-lane wave for the HIP kernels: DPP moves
// inside each row of 16 lanes (quad swaps, then the half-row and row
// mirrors, after which every lane holds its row's result) and readlane for
// the four rows.  Every lane receives the same result, formed in the same
// order in every wave, at a few cycles per step instead of the LDS round
// trip of a shuffle.  All 64 lanes must be active.
#pragma once

#include <hip/hip_runtime.h>

namespace wave {

template <int CTRL>
__device__ inline double dpp_mov(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

__device__ inline double lane_of(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// op over the 16 lanes of each row (every lane gets its row's result)
template <class Op>
__device__ inline double row16(double v, Op op) {
  v = op(v, dpp_mov<0xB1>(v));    // quad_perm [1, 0, 3, 2]
  v = op(v, dpp_mov<0x4E>(v));    // quad_perm [2, 3, 0, 1]
  v = op(v, dpp_mov<0x141>(v));   // row_half_mirror
  v = op(v, dpp_mov<0x140>(v));   // row_mirror
  return v;
}

template <class Op>
__device__ inline double all64(double v, Op op) {
  v = row16(v, op);
  return op(op(lane_of(v, 0), lane_of(v, 16)), op(lane_of(v, 32), lane_of(v, 48)));
}

__device__ inline double sum(double v) {
  return all64(v, [](double a, double b) { return a + b; });
}
__device__ inline double prod(double v) {
  return all64(v, [](double a, double b) { return a * b; });
}
__device__ inline double max(double v) {
  return all64(v, [](double a, double b) { return fmax(a, b); });
}

// sum over each group of T consecutive lanes (T a power of two <= 64); the
// groups of 32 are joined by one shuffle, smaller groups by shuffles only
__device__ inline double group_sum(double v, int T) {
  if (T == 64) return sum(v);
  if (T >= 16) {
    v = row16(v, [](double a, double b) { return a + b; });
    if (T == 32) v += __shfl_xor(v, 16);
    return v;
  }
  for (int o = T >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

}  // namespace wave
