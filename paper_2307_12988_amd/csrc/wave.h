// Wave-level (64-lane) helpers shared by the initializer and fit kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cg {

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Butterfly all-reduce: every lane ends with the same, bit-identical sum
// (each step adds the same two operands in every lane of a pair).
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

__device__ __forceinline__ int wave_count(bool pred) {
  return __popcll(__ballot(pred));
}

// Order-preserving map of float bits to unsigned (negatives below positives).
__device__ __forceinline__ uint32_t float_key(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float key_float(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

// Start point of the Lorentzian fit from one row of the 7x7-median image.
// Lane l holds row values i = l + 64 q, q < Q (masked beyond k).
//   c0 = first index of the minimum, b0 = lower median (order statistic
//   (k-1)/2), d0 = clip(1 - M[c0]/b0, 0.05, 0.95) (0.05 if b0 <= 0),
//   w0 = max(2, #{M < b0 (1 - d0/2)}); decisions in float32, IEEE rounding.
template <int Q>
__device__ __forceinline__ void start_point(const float (&mv)[Q], int k, float& c0, float& w0,
                                            float& d0, float& b0) {
  const int lane = lane_id();
  // argmin with ties to the lowest index
  float best = __builtin_inff();
  int besti = 0x7fffffff;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int i = lane + 64 * q;
    if (i < k && (mv[q] < best || (mv[q] == best && i < besti))) {
      best = mv[q];
      besti = i;
    }
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    const float ob = __shfl_xor(best, m, 64);
    const int oi = __shfl_xor(besti, m, 64);
    if (ob < best || (ob == best && oi < besti)) {
      best = ob;
      besti = oi;
    }
  }
  // radix select of the lower median on order-preserving keys
  uint32_t keys[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) keys[q] = float_key(mv[q]);
  int rank = (k - 1) / 2;
  uint32_t prefix = 0u, himask = 0u;
  for (int bit = 31; bit >= 0; --bit) {
    const uint32_t b = 1u << bit;
    int c = 0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int i = lane + 64 * q;
      const bool match = (i < k) && (((keys[q] ^ prefix) & himask) == 0u) && !(keys[q] & b);
      c += wave_count(match);
    }
    if (rank >= c) {
      prefix |= b;
      rank -= c;
    }
    himask |= b;
  }
  const float med = key_float(prefix);
  float d;
  if (med > 0.0f) {
    d = __fsub_rn(1.0f, __fdiv_rn(best, med));
    d = fminf(fmaxf(d, 0.05f), 0.95f);
  } else {
    d = 0.05f;
  }
  const float thr = __fmul_rn(med, __fsub_rn(1.0f, __fmul_rn(d, 0.5f)));
  int cnt = 0;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int i = lane + 64 * q;
    cnt += wave_count(i < k && mv[q] < thr);
  }
  c0 = (float)besti;
  w0 = (float)(cnt > 2 ? cnt : 2);
  d0 = d;
  b0 = med;
}

}  // namespace cg
