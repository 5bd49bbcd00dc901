// Wave-level (64-lane) and 16-lane-group helpers shared by the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cg {

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// ---------------------------------------------------------------------------
// DPP permutations inside a row of 16 lanes (gfx9 DPP control codes).
//   0xB1 quad_perm [1,0,3,2]  (lane ^ 1)
//   0x4E quad_perm [2,3,0,1]  (lane ^ 2)
//   0x141 row_half_mirror     (lane -> 7 - lane within each 8)
//   0x140 row_mirror          (lane -> 15 - lane within each 16)
// After the quad steps every lane of a quad holds the same value, so the two
// mirror steps pair each quad (then each half row) with its partner; each step
// adds the same two operands in both lanes of a pair, so all 16 lanes end with
// bit-identical sums.
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(dpp_i<CTRL>(__float_as_int(v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = dpp_i<CTRL>(__double2loint(v));
  const int hi = dpp_i<CTRL>(__double2hiint(v));
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ float sum16(float v) {
  v += dpp_f<0xB1>(v);
  v += dpp_f<0x4E>(v);
  v += dpp_f<0x141>(v);
  v += dpp_f<0x140>(v);
  return v;
}
__device__ __forceinline__ double sum16(double v) {
  v += dpp_d<0xB1>(v);
  v += dpp_d<0x4E>(v);
  v += dpp_d<0x141>(v);
  v += dpp_d<0x140>(v);
  return v;
}
__device__ __forceinline__ int sum16(int v) {
  v += dpp_i<0xB1>(v);
  v += dpp_i<0x4E>(v);
  v += dpp_i<0x141>(v);
  v += dpp_i<0x140>(v);
  return v;
}
// Sums over groups of 8 lanes (half rows): the two quad steps and the
// half-row mirror.
__device__ __forceinline__ float sum8(float v) {
  v += dpp_f<0xB1>(v);
  v += dpp_f<0x4E>(v);
  v += dpp_f<0x141>(v);
  return v;
}
__device__ __forceinline__ double sum8(double v) {
  v += dpp_d<0xB1>(v);
  v += dpp_d<0x4E>(v);
  v += dpp_d<0x141>(v);
  return v;
}
// Sum over a group of G lanes (G = 8 or 16), bit-identical in every lane.
template <int G>
__device__ __forceinline__ float sum_group(float v) {
  if constexpr (G == 8) return sum8(v);
  else return sum16(v);
}
template <int G>
__device__ __forceinline__ double sum_group(double v) {
  if constexpr (G == 8) return sum8(v);
  else return sum16(v);
}

__device__ __forceinline__ uint64_t min16(uint64_t v) {
#define CG_MIN_STEP(C)                                                                 \
  {                                                                                    \
    const uint32_t lo = (uint32_t)dpp_i<C>((int)(uint32_t)v);                           \
    const uint32_t hi = (uint32_t)dpp_i<C>((int)(uint32_t)(v >> 32));                   \
    const uint64_t o = ((uint64_t)hi << 32) | lo;                                      \
    v = o < v ? o : v;                                                                 \
  }
  CG_MIN_STEP(0xB1)
  CG_MIN_STEP(0x4E)
  CG_MIN_STEP(0x141)
  CG_MIN_STEP(0x140)
#undef CG_MIN_STEP
  return v;
}

__device__ __forceinline__ uint32_t min16(uint32_t v) {
  uint32_t o;
  o = (uint32_t)dpp_i<0xB1>((int)v);
  v = o < v ? o : v;
  o = (uint32_t)dpp_i<0x4E>((int)v);
  v = o < v ? o : v;
  o = (uint32_t)dpp_i<0x141>((int)v);
  v = o < v ? o : v;
  o = (uint32_t)dpp_i<0x140>((int)v);
  v = o < v ? o : v;
  return v;
}
__device__ __forceinline__ uint32_t max16(uint32_t v) {
  uint32_t o;
  o = (uint32_t)dpp_i<0xB1>((int)v);
  v = o > v ? o : v;
  o = (uint32_t)dpp_i<0x4E>((int)v);
  v = o > v ? o : v;
  o = (uint32_t)dpp_i<0x141>((int)v);
  v = o > v ? o : v;
  o = (uint32_t)dpp_i<0x140>((int)v);
  v = o > v ? o : v;
  return v;
}

// Order-preserving map of float bits to unsigned (negatives below positives).
__device__ __forceinline__ uint32_t float_key(float f) {
  const uint32_t u = __float_as_uint(f);
  // negatives: all bits flipped; others: the sign bit set
  return u ^ ((uint32_t)((int32_t)u >> 31) | 0x80000000u);
}
__device__ __forceinline__ float key_float(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

// #{q : keys[q] - base < piv} summed over a group of 16 lanes (unsigned
// differences, so keys below base wrap to large values and do not count).
// One compare and one add with carry per key, in two interleaved chains; the
// empty asm keeps the compiler from packing the comparisons into a bit mask
// and popcount.
template <int Q>
__device__ __forceinline__ int count_below16(const uint32_t (&keys)[Q], uint32_t piv,
                                             uint32_t base = 0u) {
  uint32_t ca = 0, cb = 0;
#pragma unroll
  for (int q = 0; q + 1 < Q; q += 2) {
    ca += (uint32_t)(keys[q] - base < piv);
    cb += (uint32_t)(keys[q + 1] - base < piv);
    asm volatile("" : "+v"(ca), "+v"(cb));
  }
  if constexpr (Q % 2 == 1) ca += (uint32_t)(keys[Q - 1] - base < piv);
  return sum16((int)(ca + cb));
}

// ---------------------------------------------------------------------------
// Start point of the Lorentzian fit from one row of the 7x7-median image,
// computed by a group of 16 lanes.  Lane gl of the group holds row values
// i = gl + 16 q (q < Q); slots with i >= k must hold a copy of a value of
// the row (the callers repeat the last tooth), so that the minimum, maximum
// and guess need no mask: a copy never beats its original, whose index is
// smaller.
//   c0 = first index of the minimum; b0 = lower median (order statistic
//   (k-1)/2, found by counting over order-preserving keys);
//   d0 = clip(1 - M[c0]/b0, 0.05, 0.95), 0.05 if b0 <= 0;
//   w0 = max(2, #{M < b0 (1 - d0/2)}).
// The arithmetic that decides d0 and the count uses IEEE float32 operations in
// that order (no contraction), so identical inputs give identical results.
// The start centre alone: the first index of the smallest filtered value,
// as start_point16 finds it (same keys, same tie rule).
template <int Q>
__device__ __forceinline__ float start_centre16(const float (&mv)[Q]) {
  const int gl = lane_id() & 15;
  uint32_t bk = 0xffffffffu, bi = 0u;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const uint32_t key = float_key(mv[q] + 0.0f);  // -0 -> +0
    const bool lt = key < bk || q == 0;
    bk = lt ? key : bk;
    bi = lt ? (uint32_t)(gl + 16 * q) : bi;
  }
  const uint64_t best = min16(((uint64_t)bk << 32) | bi);
  return (float)(int)(uint32_t)best;
}

template <int Q>
__device__ __forceinline__ void start_point16(const float (&mv)[Q], int k, float& c0, float& w0,
                                              float& d0, float& b0) {
  const int gl = lane_id() & 15;
  uint32_t keys[Q];
  // the lane's first minimum (slots in increasing index), then the group's
  uint32_t bk = 0xffffffffu, bi = 0u;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    keys[q] = float_key(mv[q] + 0.0f);  // -0 -> +0: equal values, equal keys
    const bool lt = keys[q] < bk || q == 0;
    bk = lt ? keys[q] : bk;
    bi = lt ? (uint32_t)(gl + 16 * q) : bi;
  }
  const uint64_t best = min16(((uint64_t)bk << 32) | bi);
  const int besti = (int)(uint32_t)best;
  const float bestv = key_float((uint32_t)(best >> 32));

  // Lower median (order statistic r = (k-1)/2).  The key interval [lo, hi]
  // always holds it, with c_lo = #{keys < lo} <= r < c_hi = #{keys <= hi};
  // every probe lies in (lo, hi], so the choice of probes changes only how
  // fast the interval shrinks, never the result.  A gallop from a guess and
  // then bisection shrink it until at most four keys lie in it; the
  // remaining keys are then taken in order, smallest first, until the count
  // passes r.  (Near the median the keys are dense, so isolating a single
  // key by bisection takes several more probes than reading the last few.)
  const int r = (k - 1) / 2;
  uint32_t lo = (uint32_t)(best >> 32), hi = 0u;
#pragma unroll
  for (int q = 0; q < Q; ++q) hi = keys[q] > hi ? keys[q] : hi;
  hi = max16(hi);
  // Teeth past the end take the largest key: no key is below it and no
  // probe above it, so they never count and the counts need no mask.
#pragma unroll
  for (int q = 0; q < Q; ++q) keys[q] = gl + 16 * q < k ? keys[q] : 0xffffffffu;
  int c_lo = 0, c_hi = k;
  if (lo < hi && c_hi - c_lo > 4) {
    // Gallop from a guess, the mean of the values at or above the row mean
    // (the dip pulls the plain mean below the baseline), in steps that double
    // until they leave [lo, hi]; this skips most of the probes that bisection
    // from [min, max] spends outside the baseline cluster.  The repeated last
    // tooth takes part in the guess: it moves the guess, not the result.
    float sm = 0.0f;
#pragma unroll
    for (int q = 0; q < Q; ++q) sm += mv[q];
    sm = sum16(sm);
    const float mean = sm * (1.0f / (16 * Q));
    float su = 0.0f;
    int nu = 0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const bool up = mv[q] >= mean;
      su += up ? mv[q] : 0.0f;
      nu += up ? 1 : 0;
    }
    su = sum16(su);  // bit-identical in the 16 lanes, so the probes are too
    nu = sum16(nu);
    uint32_t mid = float_key(su * __builtin_amdgcn_rcpf((float)(nu > 0 ? nu : 1)) + 0.0f);
    mid = mid <= lo ? lo + 1u : (mid > hi ? hi : mid);
    uint32_t step = (hi - lo) >> 8;
    step = step > 0u ? step : 1u;
    for (int p = 0; p < 10 && c_hi - c_lo > 4; ++p) {
      const int c = count_below16(keys, mid);
      if (c <= r) {
        lo = mid;
        c_lo = c;
        if (hi - mid < step) break;
        mid += step;  // still <= hi
      } else {
        hi = mid - 1u;
        c_hi = c;
        if (mid - lo <= step) break;
        mid -= step;  // still > lo
      }
      step = step < 0x40000000u ? step << 1 : step;
    }
  }
  while (lo < hi && c_hi - c_lo > 4) {
    const uint32_t mid = lo + ((hi - lo) >> 1) + 1u;  // lo < mid <= hi
    const int c = count_below16(keys, mid);
    if (c <= r) {
      lo = mid;
      c_lo = c;
    } else {
      hi = mid - 1u;
      c_hi = c;
    }
  }
  if (lo < hi) {
    // Each round finds the smallest key m >= cur (keys below cur wrap to
    // large differences) and counts the keys in [cur, m]; the answer is the
    // first m at which the count passes r.  At most four distinct keys
    // remain, so at most four rounds.
    uint32_t cur = lo, m = lo;
    int c = c_lo;
    for (int e = 0; e < 4; ++e) {
      uint32_t dmin = 0xffffffffu;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const uint32_t dq = keys[q] - cur;
        dmin = dq < dmin ? dq : dmin;
      }
      dmin = min16(dmin);
      m = cur + dmin;  // dmin + 1 does not wrap: a key <= hi < 2^32 - 1 is >= cur
      c += count_below16(keys, dmin + 1u, cur);
      if (c > r) break;
      cur = m + 1u;
    }
    lo = m;
  }
  const uint32_t prefix = lo;
  const float med = key_float(prefix);
  float d;
  if (med > 0.0f) {
    d = __fsub_rn(1.0f, __fdiv_rn(bestv, med));
    d = fminf(fmaxf(d, 0.05f), 0.95f);
  } else {
    d = 0.05f;
  }
  const float thr = __fmul_rn(med, __fsub_rn(1.0f, __fmul_rn(d, 0.5f)));
  // M < thr compared as keys (the same order for non-NaN values; the slots
  // past the end carry the largest key and never count)
  const int cnt = count_below16(keys, float_key(thr + 0.0f));
  c0 = (float)besti;
  w0 = (float)(cnt > 2 ? cnt : 2);
  d0 = d;
  b0 = med;
}

// Dispatch a runtime tooth count to the smallest per-lane slot count that
// covers it with 16 lanes: Q in {1, 2, 4, 8, 14, 20, 28} (k <= 16 .. 448).
#define CG_DISPATCH_Q16(k, CALL)        \
  do {                                   \
    const int _k = (k);                  \
    if (_k <= 16) {                      \
      constexpr int Q = 1;               \
      CALL;                              \
    } else if (_k <= 32) {               \
      constexpr int Q = 2;               \
      CALL;                              \
    } else if (_k <= 64) {               \
      constexpr int Q = 4;               \
      CALL;                              \
    } else if (_k <= 128) {              \
      constexpr int Q = 8;               \
      CALL;                              \
    } else if (_k <= 224) {              \
      constexpr int Q = 14;              \
      CALL;                              \
    } else if (_k <= 320) {              \
      constexpr int Q = 20;              \
      CALL;                              \
    } else {                             \
      constexpr int Q = 28;              \
      CALL;                              \
    }                                    \
  } while (0)

}  // namespace cg
