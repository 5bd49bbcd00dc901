// Tooth DFT as a dense contraction on the matrix cores (precision form).
//
// The comb-tooth amplitudes need the DFT only at the K tooth bins, which is a
// dense product of the frames [F x N] with the basis [N x 2K] whose columns are
// cos(2 pi k_i t / N) and -sin(2 pi k_i t / N).  On gfx950 it runs on
// v_mfma_f32_16x16x32_{bf16,f16} with FP32 accumulation, in three forms:
//
//   BF16X3  x = x_hi + x_lo exactly: x_hi keeps the 8 leading significant bits
//           of x (bf16 truncation), x_lo = x - x_hi has at most 8 significant
//           bits and |x_lo| < 2^-7 |x|; W = W_hi + W_lo (bf16 rounding of W and
//           of the FP64 remainder).  Sum x_hi W_hi + x_hi W_lo + x_lo W_hi; the
//           dropped x_lo W_lo is below 2^-16 |x W|.
//   FP16    x and W rounded to fp16; one product.
//   FP16X2  x = x_hi + x_lo exactly (low 5 bits split off, both exact in
//           fp16), W rounded to fp16; two products.
//
// Epilogue: amplitude sqrt(re^2 + im^2) and division by the reference, the
// same outputs as the FFT path.  The basis is built on the host in FP64 from
// the integer phase index (k t mod N) and rounded once.
//
// Tiling: a 256-thread block computes 128 frames x 64 teeth (cos and sin
// accumulators for each); each wave takes 32 frames x 64 teeth, i.e. 2 x 4
// MFMA tiles of 16 x 16, for both the cos and the sin columns.  Each step of 32
// samples stages the frames (converted to the operand format) and the basis
// slices in LDS; the next step's global loads are issued before the current
// step's MFMAs.  Blocks of the same frame rows are adjacent in launch order so
// the frames are read from HBM about once and re-used from L2 by the tooth
// blocks.
#include <cmath>
#include <cstring>

#include "internal.h"

namespace cg {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

constexpr int BM = 128;      // frames per block
constexpr int BT = 64;       // teeth per block
constexpr int KS = 32;       // samples per step
constexpr int PITCH = 40;    // LDS row pitch in 16-bit elements (80 B, 16-B aligned)

__device__ __forceinline__ uint16_t bf16_bits_exact(float f) {
  return (uint16_t)(__float_as_uint(f) >> 16);  // exact for values with <= 8 significant bits
}
__device__ __forceinline__ uint16_t f16_bits(float f) {
  _Float16 h = (_Float16)f;
  return __builtin_bit_cast(uint16_t, h);
}

template <int FORM>
__global__ __launch_bounds__(256) void mfma_teeth_kernel(
    const int16_t* __restrict__ frames, int64_t nf, int n, int k, int tooth_blocks,
    const uint16_t* __restrict__ bc_hi, const uint16_t* __restrict__ bc_lo,
    const uint16_t* __restrict__ bs_hi, const uint16_t* __restrict__ bs_lo,
    const float* __restrict__ ref, float* __restrict__ out_mag, float* __restrict__ out_y) {
  constexpr bool SPLIT_A = FORM != 1;       // BF16X3, FP16X2
  constexpr bool SPLIT_B = FORM == 0;       // BF16X3
  __shared__ __attribute__((aligned(16))) uint16_t sa_hi[BM * PITCH];
  __shared__ __attribute__((aligned(16))) uint16_t sa_lo[SPLIT_A ? BM * PITCH : 8];
  __shared__ __attribute__((aligned(16))) uint16_t sc_hi[BT * PITCH];
  __shared__ __attribute__((aligned(16))) uint16_t ss_hi[BT * PITCH];
  __shared__ __attribute__((aligned(16))) uint16_t sc_lo[SPLIT_B ? BT * PITCH : 8];
  __shared__ __attribute__((aligned(16))) uint16_t ss_lo[SPLIT_B ? BT * PITCH : 8];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave;
  const int tb = blockIdx.x % tooth_blocks;
  const int64_t f0 = (int64_t)(blockIdx.x / tooth_blocks) * BM;
  const int t0 = tb * BT;
  const int kpad = tooth_blocks * BT;

  // staging assignment: each thread moves 8 consecutive samples of two frame
  // rows (srow, srow + 64) and of one basis row (srow)
  const int srow = tid >> 2;
  const int scol = (tid & 3) * 8;
  const int64_t frow0 = f0 + srow, frow1 = f0 + 64 + srow;
  const bool ok0 = frow0 < nf, ok1 = frow1 < nf;
  const int16_t* a_src0 = frames + (ok0 ? frow0 : 0) * (int64_t)n + scol;
  const int16_t* a_src1 = frames + (ok1 ? frow1 : 0) * (int64_t)n + scol;
  const size_t b_off = (size_t)(t0 + srow) * n + scol;

  f32x4 acc_c[2][4], acc_s[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      acc_c[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
      acc_s[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    }

  const u16x8 zero8 = {0, 0, 0, 0, 0, 0, 0, 0};
  u16x8 ra0, ra1, rbch, rbsh, rbcl, rbsl;
  auto gload = [&](int s0) {
    ra0 = ok0 ? *reinterpret_cast<const u16x8*>(a_src0 + s0) : zero8;
    ra1 = ok1 ? *reinterpret_cast<const u16x8*>(a_src1 + s0) : zero8;
    rbch = *reinterpret_cast<const u16x8*>(bc_hi + b_off + s0);
    rbsh = *reinterpret_cast<const u16x8*>(bs_hi + b_off + s0);
    if constexpr (SPLIT_B) {
      rbcl = *reinterpret_cast<const u16x8*>(bc_lo + b_off + s0);
      rbsl = *reinterpret_cast<const u16x8*>(bs_lo + b_off + s0);
    }
  };
  auto convert = [&](const u16x8& ra, u16x8& hi, u16x8& lo) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int x = (int)(int16_t)ra[j];
      if constexpr (FORM == 0) {
        const float xf = (float)x;
        const float xh = __uint_as_float(__float_as_uint(xf) & 0xffff0000u);
        hi[j] = bf16_bits_exact(xh);
        lo[j] = bf16_bits_exact(xf - xh);
      } else if constexpr (FORM == 1) {
        hi[j] = f16_bits((float)x);
      } else {
        const int xh = x & ~0x1f;
        hi[j] = f16_bits((float)xh);
        lo[j] = f16_bits((float)(x - xh));
      }
    }
  };
  auto lstore = [&]() {
    u16x8 hi, lo;
    convert(ra0, hi, lo);
    *reinterpret_cast<u16x8*>(sa_hi + srow * PITCH + scol) = hi;
    if constexpr (SPLIT_A) *reinterpret_cast<u16x8*>(sa_lo + srow * PITCH + scol) = lo;
    convert(ra1, hi, lo);
    *reinterpret_cast<u16x8*>(sa_hi + (64 + srow) * PITCH + scol) = hi;
    if constexpr (SPLIT_A) *reinterpret_cast<u16x8*>(sa_lo + (64 + srow) * PITCH + scol) = lo;
    *reinterpret_cast<u16x8*>(sc_hi + srow * PITCH + scol) = rbch;
    *reinterpret_cast<u16x8*>(ss_hi + srow * PITCH + scol) = rbsh;
    if constexpr (SPLIT_B) {
      *reinterpret_cast<u16x8*>(sc_lo + srow * PITCH + scol) = rbcl;
      *reinterpret_cast<u16x8*>(ss_lo + srow * PITCH + scol) = rbsl;
    }
  };

  const int fr = lane & 15;          // operand row / column within a 16x16 tile
  const int kq = (lane >> 4) * 8;    // operand k offset
  gload(0);
  for (int s0 = 0; s0 < n; s0 += KS) {
    __syncthreads();
    lstore();
    __syncthreads();
    if (s0 + KS < n) gload(s0 + KS);
    u16x8 ah[2], al[2], ch[4], sh[4], cl[4], sl[4];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int row = wr * 32 + i * 16 + fr;
      ah[i] = *reinterpret_cast<const u16x8*>(sa_hi + row * PITCH + kq);
      if constexpr (SPLIT_A) al[i] = *reinterpret_cast<const u16x8*>(sa_lo + row * PITCH + kq);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = j * 16 + fr;
      ch[j] = *reinterpret_cast<const u16x8*>(sc_hi + col * PITCH + kq);
      sh[j] = *reinterpret_cast<const u16x8*>(ss_hi + col * PITCH + kq);
      if constexpr (SPLIT_B) {
        cl[j] = *reinterpret_cast<const u16x8*>(sc_lo + col * PITCH + kq);
        sl[j] = *reinterpret_cast<const u16x8*>(ss_lo + col * PITCH + kq);
      }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if constexpr (FORM == 0) {
          const bf16x8 a1 = __builtin_bit_cast(bf16x8, ah[i]);
          const bf16x8 a2 = __builtin_bit_cast(bf16x8, al[i]);
          const bf16x8 c1 = __builtin_bit_cast(bf16x8, ch[j]);
          const bf16x8 c2 = __builtin_bit_cast(bf16x8, cl[j]);
          const bf16x8 s1 = __builtin_bit_cast(bf16x8, sh[j]);
          const bf16x8 s2 = __builtin_bit_cast(bf16x8, sl[j]);
          acc_c[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, c1, acc_c[i][j], 0, 0, 0);
          acc_c[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, c2, acc_c[i][j], 0, 0, 0);
          acc_c[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, c1, acc_c[i][j], 0, 0, 0);
          acc_s[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, s1, acc_s[i][j], 0, 0, 0);
          acc_s[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, s2, acc_s[i][j], 0, 0, 0);
          acc_s[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, s1, acc_s[i][j], 0, 0, 0);
        } else {
          const f16x8 a1 = __builtin_bit_cast(f16x8, ah[i]);
          const f16x8 c1 = __builtin_bit_cast(f16x8, ch[j]);
          const f16x8 s1 = __builtin_bit_cast(f16x8, sh[j]);
          acc_c[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a1, c1, acc_c[i][j], 0, 0, 0);
          acc_s[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a1, s1, acc_s[i][j], 0, 0, 0);
          if constexpr (FORM == 2) {
            const f16x8 a2 = __builtin_bit_cast(f16x8, al[i]);
            acc_c[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a2, c1, acc_c[i][j], 0, 0, 0);
            acc_s[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a2, s1, acc_s[i][j], 0, 0, 0);
          }
        }
      }
  }
  // epilogue: lane holds rows 4*(lane/16)+e of each 16x16 tile, column lane%16
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int tooth = t0 + j * 16 + fr;
      if (tooth >= k) continue;
      const float rf = ref[tooth];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t f = f0 + wr * 32 + i * 16 + (lane >> 4) * 4 + e;
        if (f >= nf) continue;
        const float re = acc_c[i][j][e], im = acc_s[i][j][e];
        const float mag = sqrtf(re * re + im * im);
        if (out_mag) out_mag[f * k + tooth] = mag;
        if (out_y) out_y[f * k + tooth] = mag / rf;
      }
    }
  (void)kpad;
}

}  // namespace

cg_status mfma_prepare(cg_plan* p, uint32_t form) {
  const bool bf = form == CG_DFT_MFMA_BF16X3;
  uint16_t*& slot0 = bf ? p->d_mfma_bf[0] : p->d_mfma_h[0];
  if (slot0) return CG_OK;
  const int n = p->n;
  const int kpad = ((p->k + 63) / 64) * 64;
  const size_t elems = (size_t)kpad * n;
  std::vector<uint16_t> h[4];
  const int nmat = bf ? 4 : 2;
  for (int m = 0; m < nmat; ++m) h[m].assign(elems, 0);
  auto to_bf16 = [](double v) {  // round to nearest even
    const float f = (float)v;
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
  };
  auto bf16_val = [](uint16_t b) {
    const uint32_t u = (uint32_t)b << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return (double)f;
  };
  for (int i = 0; i < p->k; ++i) {
    const int64_t kb = p->h_bins[i];
    for (int t = 0; t < n; ++t) {
      const int64_t ph = (kb * t) % n;
      const double a = 2.0 * (double)ph / (double)n;  // angle / pi
      const double c = std::cos(M_PI * a), s = -std::sin(M_PI * a);
      const size_t o = (size_t)i * n + t;
      if (bf) {
        h[0][o] = to_bf16(c);
        h[1][o] = to_bf16(c - bf16_val(h[0][o]));
        h[2][o] = to_bf16(s);
        h[3][o] = to_bf16(s - bf16_val(h[2][o]));
      } else {
        const _Float16 hc = (_Float16)c, hs = (_Float16)s;
        std::memcpy(&h[0][o], &hc, 2);
        std::memcpy(&h[1][o], &hs, 2);
      }
    }
  }
  for (int m = 0; m < nmat; ++m) {
    uint16_t*& dst = bf ? p->d_mfma_bf[m] : p->d_mfma_h[m];
    hipError_t e = hipMalloc(&dst, elems * sizeof(uint16_t));
    if (e == hipSuccess)
      e = hipMemcpy(dst, h[m].data(), elems * sizeof(uint16_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "MFMA basis");
  }
  return CG_OK;
}

hipError_t launch_mfma_teeth(const cg_plan* p, uint32_t form, const int16_t* frames, int64_t nf,
                             float* out_mag, float* out_y, hipStream_t s) {
  const int tooth_blocks = (p->k + BT - 1) / BT;
  const int64_t blocks = ((nf + BM - 1) / BM) * tooth_blocks;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 g((unsigned)blocks), b(256);
  switch (form) {
    case CG_DFT_MFMA_BF16X3:
      hipLaunchKernelGGL(mfma_teeth_kernel<0>, g, b, 0, s, frames, nf, p->n, p->k, tooth_blocks,
                         p->d_mfma_bf[0], p->d_mfma_bf[1], p->d_mfma_bf[2], p->d_mfma_bf[3],
                         p->d_ref, out_mag, out_y);
      break;
    case CG_DFT_MFMA_FP16:
      hipLaunchKernelGGL(mfma_teeth_kernel<1>, g, b, 0, s, frames, nf, p->n, p->k, tooth_blocks,
                         p->d_mfma_h[0], nullptr, p->d_mfma_h[1], nullptr, p->d_ref, out_mag,
                         out_y);
      break;
    case CG_DFT_MFMA_FP16X2:
      hipLaunchKernelGGL(mfma_teeth_kernel<2>, g, b, 0, s, frames, nf, p->n, p->k, tooth_blocks,
                         p->d_mfma_h[0], nullptr, p->d_mfma_h[1], nullptr, p->d_ref, out_mag,
                         out_y);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace cg
