// Learned warm start: a 220 -> 256 -> 256 -> 4 network (GELU) that maps a
// normalised tooth vector to standardised start parameters (c, w, d, b) of the
// Lorentzian fit, with the project's own training kernels.
//
// Precision: matrix products take bfloat16 operands (round to nearest even)
// on v_mfma_f32_16x16x32_bf16 with FP32 accumulation; biases, GELU (exact erf),
// the loss and Adam run in FP32; master weights and Adam moments are FP32.
//
// Kernels
// -------
// * gemm_kernel<LA, LB>: C[m][n] = sum_k A(m,k) B(n,k) for bf16 A and B given
//   by strides (either k or the row index contiguous), 64 x 64 tiles, four
//   waves of 2 x 2 MFMA tiles, K steps of 32 staged in LDS, every load
//   bounds-checked (zero fill), epilogues: store (+ bias), bias + GELU
//   (keeps the pre-activation for backward and writes the bf16 activation),
//   GELU backward (dH = dA * GELU'(H), FP32 and bf16 copies).
// * column sums (bias gradients), loss + dOut, Adam, bf16 weight refresh, a
//   row gather for mini-batches.
// * mlp_infer_kernel: the whole forward pass for 64 frames per block with the
//   activations in LDS (never in HBM), input resampled to 220 points when
//   K != 220, output de-standardised and rescaled to the tooth axis.
#include <cmath>
#include <cstring>

#include "internal.h"
#include "mlp.h"

namespace cg {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

constexpr float kInvSqrt2 = 0.70710678118654752f;
constexpr float kInvSqrt2Pi = 0.39894228040143268f;

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * kInvSqrt2)); }
__device__ __forceinline__ float gelu_grad(float z) {
  const float cdf = 0.5f * (1.0f + erff(z * kInvSqrt2));
  return cdf + z * kInvSqrt2Pi * expf(-0.5f * z * z);
}

constexpr int TM = 64, TN = 64, TK = 32, LP = 40;  // tile, LDS pitch (bf16 elements)

enum Epi : int { EPI_STORE = 0, EPI_GELU = 1, EPI_DGELU = 2 };

struct GemmEpi {
  int mode;
  const float* bias;  // [N] (store / gelu)
  float* c;           // fp32 out [M][ldc]: plain result, pre-activation, or dH
  int ldc;
  uint16_t* cb;       // bf16 out [M][ldcb]: activation or dH (gelu / dgelu)
  int ldcb;
  const float* hin;   // pre-activation for GELU backward [M][ldh]
  int ldh;
};

// LA == 0: A(m,k) = A[m * lda + k]   LA == 1: A(m,k) = A[k * lda + m]
template <int LA, int LB>
__global__ __launch_bounds__(256) void gemm_kernel(int M, int N, int K,
                                                   const uint16_t* __restrict__ A, int lda,
                                                   const uint16_t* __restrict__ B, int ldb,
                                                   GemmEpi ep) {
  __shared__ __attribute__((aligned(16))) uint16_t sa[TM * LP];
  __shared__ __attribute__((aligned(16))) uint16_t sb[TN * LP];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave & 1, wc = wave >> 1;
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int fr = lane & 15, kq = (lane >> 4) * 8;
  for (int k0 = 0; k0 < K; k0 += TK) {
    __syncthreads();
    // stage 64 x 32 of A and of B (8 elements per thread each)
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      int r, kk;
      if (LA == 0) {
        r = tid >> 2;
        kk = (tid & 3) * 8 + e;
      } else {
        kk = tid >> 3;
        r = (tid & 7) * 8 + e;
      }
      const int m = m0 + r, k = k0 + kk;
      uint16_t v = 0;
      if (m < M && k < K) v = LA == 0 ? A[(size_t)m * lda + k] : A[(size_t)k * lda + m];
      sa[r * LP + kk] = v;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      int r, kk;
      if (LB == 0) {
        r = tid >> 2;
        kk = (tid & 3) * 8 + e;
      } else {
        kk = tid >> 3;
        r = (tid & 7) * 8 + e;
      }
      const int n = n0 + r, k = k0 + kk;
      uint16_t v = 0;
      if (n < N && k < K) v = LB == 0 ? B[(size_t)n * ldb + k] : B[(size_t)k * ldb + n];
      sb[r * LP + kk] = v;
    }
    __syncthreads();
    u16x8 af[2], bfr[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      af[i] = *reinterpret_cast<const u16x8*>(sa + (wr * 32 + i * 16 + fr) * LP + kq);
      bfr[i] = *reinterpret_cast<const u16x8*>(sb + (wc * 32 + i * 16 + fr) * LP + kq);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, af[i]),
                                                            __builtin_bit_cast(bf16x8, bfr[j]),
                                                            acc[i][j], 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int n = n0 + wc * 32 + j * 16 + fr;
      if (n >= N) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int m = m0 + wr * 32 + i * 16 + (lane >> 4) * 4 + e;
        if (m >= M) continue;
        float v = acc[i][j][e];
        if (ep.mode == EPI_STORE) {
          if (ep.bias) v += ep.bias[n];
          ep.c[(size_t)m * ep.ldc + n] = v;
        } else if (ep.mode == EPI_GELU) {
          v += ep.bias[n];
          if (ep.c) ep.c[(size_t)m * ep.ldc + n] = v;
          ep.cb[(size_t)m * ep.ldcb + n] = to_bf16(gelu(v));
        } else {
          const float d = v * gelu_grad(ep.hin[(size_t)m * ep.ldh + n]);
          if (ep.c) ep.c[(size_t)m * ep.ldc + n] = d;
          ep.cb[(size_t)m * ep.ldcb + n] = to_bf16(d);
        }
      }
    }
}

template <int LA, int LB>
hipError_t gemm(int M, int N, int K, const uint16_t* A, int lda, const uint16_t* B, int ldb,
                const GemmEpi& ep, hipStream_t s) {
  dim3 g((N + TN - 1) / TN, (M + TM - 1) / TM);
  hipLaunchKernelGGL((gemm_kernel<LA, LB>), g, dim3(256), 0, s, M, N, K, A, lda, B, ldb, ep);
  return hipGetLastError();
}

// out[j] (+)= sum_r x[r * ld + j], r < rows, in row order (deterministic)
__global__ void colsum_kernel(const float* __restrict__ x, int rows, int cols, int ld,
                              float* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cols) return;
  float acc = 0.f;
  for (int r = 0; r < rows; ++r) acc += x[(size_t)r * ld + j];
  out[j] = acc;
}

// weighted MSE over [B][4]: dout = 2 w (out - t) / (4 sum w); loss (device
// scalar) written by one block of 256 threads, in a fixed reduction order
__global__ __launch_bounds__(256) void loss_kernel(const float* __restrict__ out,
                                                   const float* __restrict__ t,
                                                   const float* __restrict__ w, int b,
                                                   float* __restrict__ dout,
                                                   uint16_t* __restrict__ doutb,
                                                   float* __restrict__ loss) {
  __shared__ float s_w[256], s_l[256];
  const int tid = threadIdx.x;
  float sw = 0.f;
  for (int r = tid; r < b; r += 256) sw += w ? w[r] : 1.f;
  s_w[tid] = sw;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st) s_w[tid] += s_w[tid + st];
    __syncthreads();
  }
  const float denom = 4.f * s_w[0];
  float sl = 0.f;
  for (int r = tid; r < b; r += 256) {
    const float wr = w ? w[r] : 1.f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float d = out[r * 4 + j] - t[r * 4 + j];
      const float g = denom > 0.f ? 2.f * wr * d / denom : 0.f;
      dout[r * 4 + j] = g;
      doutb[r * 4 + j] = to_bf16(g);
      sl += wr * d * d;
    }
  }
  s_l[tid] = sl;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st) s_l[tid] += s_l[tid + st];
    __syncthreads();
  }
  if (tid == 0 && loss) *loss = denom > 0.f ? s_l[0] / denom : 0.f;
}

__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, int n, float lr,
                            float b1, float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void to_bf16_kernel(const float* __restrict__ x, uint16_t* __restrict__ y, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = to_bf16(x[i]);
}

// mini-batch gather: rows idx[r] of x [*][220] (bf16), t [*][4], w [*]
__global__ void gather_kernel(const float* __restrict__ x, const float* __restrict__ t,
                              const float* __restrict__ w, const int32_t* __restrict__ idx,
                              int b, uint16_t* __restrict__ xb, float* __restrict__ tb,
                              float* __restrict__ wb) {
  const int r = blockIdx.x;
  if (r >= b) return;
  const int64_t src = idx[r];
  for (int j = threadIdx.x; j < MLP_IN; j += blockDim.x)
    xb[(size_t)r * MLP_IN + j] = to_bf16(x[src * MLP_IN + j]);
  if (threadIdx.x < 4) tb[r * 4 + threadIdx.x] = t[src * 4 + threadIdx.x];
  if (threadIdx.x == 0) wb[r] = w ? w[src] : 1.f;
}

// ---------------------------------------------------------------------------
// GELU for inference.  erf from Abramowitz & Stegun 7.1.26 (Hastings): with
// t = 1 / (1 + p |x|), erf|x| = 1 - t (a1 + t (a2 + t (a3 + t (a4 + t a5))))
// exp(-x^2), absolute error at most 1.5e-7 -- far below the bf16 rounding
// the activations get next, and a third of the instructions of erff.
__device__ __forceinline__ float gelu_fast(float z) {
  const float x = z * kInvSqrt2;
  const float ax = fabsf(x);
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, ax, 1.0f));
  float poly = fmaf(t, 1.061405429f, -1.453152027f);
  poly = fmaf(t, poly, 1.421413741f);
  poly = fmaf(t, poly, -0.284496736f);
  poly = fmaf(t, poly, 0.254829592f);
  poly *= t;
  const float e = __builtin_amdgcn_exp2f(-1.4426950408889634f * ax * ax);  // exp(-x^2)
  const float erf_abs = fmaf(-poly, e, 1.0f);
  const float erf_x = __builtin_copysignf(erf_abs, x);
  const float h = 0.5f * z;
  return fmaf(h, erf_x, h);
}

// fused inference: 64 frames per block, activations in LDS
constexpr int IB = 64;               // frames per block
constexpr int HP = MLP_HID + 8;      // LDS pitch of hidden activations (264)

// One dense layer + bias + GELU for the block's 64 frames: wave w computes all
// 64 rows of hidden units 64 w .. 64 w + 63 (4 x 4 tiles of 16 x 16).  The
// weight fragments stream from L2 (each block reads every weight once), two
// k-steps ahead of the products that use them, so a step waits for a load
// issued two steps earlier rather than for a full round trip.
template <int KDIM>
__device__ __forceinline__ void dense_gelu64(const uint16_t* in, int pitch,
                                             const uint16_t* __restrict__ w,
                                             const float* __restrict__ bias, uint16_t* outb,
                                             int wave, int lane) {
  constexpr int NK = KDIM / 32;
  const int fr = lane & 15, kq = (lane >> 4) * 8;
  f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const uint16_t* wrow = w + (size_t)(wave * 64 + fr) * KDIM + kq;
  u16x8 wb[3][4];
  auto load_w = [&](u16x8(&wf)[4], int step) __attribute__((always_inline)) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
      wf[j] = *reinterpret_cast<const u16x8*>(wrow + (size_t)j * 16 * KDIM + step * 32);
  };
  load_w(wb[0], 0);
  if constexpr (NK > 1) load_w(wb[1], 1);
#pragma unroll
  for (int st = 0; st < NK; ++st) {
    if (st + 2 < NK) load_w(wb[(st + 2) % 3], st + 2);
    u16x8 af[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
      af[i] = *reinterpret_cast<const u16x8*>(in + (i * 16 + fr) * pitch + st * 32 + kq);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, af[i]),
                                                            __builtin_bit_cast(bf16x8, wb[st % 3][j]),
                                                            acc[i][j], 0, 0, 0);
  }
  __syncthreads();  // every wave has read `in` before `outb` (may alias) is written
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int n = wave * 64 + j * 16 + fr;
    const float bn = bias[n];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = i * 16 + (lane >> 4) * 4 + e;
        outb[r * HP + n] = to_bf16(gelu_fast(acc[i][j][e] + bn));
      }
  }
  __syncthreads();
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) void mlp_infer_kernel(
    const float* __restrict__ y, int64_t nf, int k, const uint16_t* __restrict__ w1,
    const float* __restrict__ b1, const uint16_t* __restrict__ w2, const float* __restrict__ b2,
    const uint16_t* __restrict__ w3, const float* __restrict__ b3, MlpScale sc,
    float* __restrict__ p0, const int32_t* __restrict__ dev_n) {
  // one activation buffer: each layer reads all of it before the barrier in
  // dense_gelu64 and overwrites it after (34 KB per block)
  __shared__ __attribute__((aligned(16))) uint16_t s_x[IB * HP];
  __shared__ float s_out[IB * 4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t f0 = (int64_t)blockIdx.x * IB;
  if (dev_n) {
    const int64_t dn = *dev_n;
    nf = dn < nf ? dn : nf;
  }
  if (f0 >= nf) return;
  const int fr = lane & 15, kq = (lane >> 4) * 8;

  // input: resample to 220 points when k != 220, round to bf16, zero pad.
  // Thread tid takes the values tid + 256 m of the block's 64 x 220 inputs
  // (row r, column j kept incrementally), eleven at a time so that their
  // loads are in flight together; rows past the batch repeat its last frame.
  {
    static_assert(IB * MLP_IN % 256 == 0, "whole values per thread");
    constexpr int NE = IB * MLP_IN / 256;  // 55
    const int r0 = tid / MLP_IN, j0 = tid - r0 * MLP_IN;
    const int64_t last = nf - 1;
    auto walk = [&](auto value) __attribute__((always_inline)) {
      int r = r0, j = j0;
#pragma unroll 11
      for (int m = 0; m < NE; ++m) {
        int64_t f = f0 + r;
        f = f < last ? f : last;
        s_x[r * HP + j] = to_bf16(value(f, j));
        // next value: index + 256 = (r + 1) 220 + j + 36
        j += 256 - MLP_IN;
        r += 1;
        if (j >= MLP_IN) {
          j -= MLP_IN;
          r += 1;
        }
      }
    };
    if (k == MLP_IN) {
      walk([&](int64_t f, int j) { return y[f * k + j]; });
    } else {
      // position j (k - 1) / 219 split exactly into its integer part and
      // remainder, so the interpolation weight carries one rounding only
      walk([&](int64_t f, int j) {
        const int q = j * (k - 1);
        int lo = q / (MLP_IN - 1);
        const float t = (float)(q - lo * (MLP_IN - 1)) / (float)(MLP_IN - 1);
        lo = lo > k - 1 ? k - 1 : lo;
        const int hi = lo + 1 < k ? lo + 1 : k - 1;
        return y[f * k + lo] * (1.f - t) + y[f * k + hi] * t;
      });
    }
    s_x[(tid >> 2) * HP + MLP_IN + (tid & 3)] = 0;  // columns 220 .. 223
  }
  __syncthreads();
  dense_gelu64<MLP_IN_PAD>(s_x, HP, w1, b1, s_x, wave, lane);
  dense_gelu64<MLP_HID>(s_x, HP, w2, b2, s_x, wave, lane);
  // layer 3 (256 -> 4, padded to one 16-column tile): wave w takes rows 16 w .. 16 w + 15;
  // its eight weight fragments are loaded together
  {
    f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
    u16x8 w3f[MLP_HID / 32];
#pragma unroll
    for (int st = 0; st < MLP_HID / 32; ++st)
      w3f[st] = *reinterpret_cast<const u16x8*>(w3 + (size_t)fr * MLP_HID + st * 32 + kq);
#pragma unroll
    for (int k0 = 0; k0 < MLP_HID; k0 += 32) {
      const u16x8 wf = w3f[k0 / 32];
      const u16x8 af = *reinterpret_cast<const u16x8*>(s_x + (wave * 16 + fr) * HP + k0 + kq);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, af),
                                                    __builtin_bit_cast(bf16x8, wf), acc, 0, 0, 0);
    }
    if (fr < 4) {
#pragma unroll
      for (int e = 0; e < 4; ++e) s_out[(wave * 16 + (lane >> 4) * 4 + e) * 4 + fr] = acc[e] + b3[fr];
    }
  }
  __syncthreads();
  {
    const int r = tid >> 2, j = tid & 3;
    const int64_t f = f0 + r;
    if (f < nf) {
      float v = s_out[r * 4 + j] * sc.std[j] + sc.mean[j];
      if (j < 2) v *= (float)(k - 1) / (float)(MLP_IN - 1);
      p0[f * 4 + j] = v;
    }
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// host side

static hipError_t upload_bf16(const float* host, int rows, int cols, int ld_dev, uint16_t** dev) {
  std::vector<uint16_t> h((size_t)rows * ld_dev, 0);
  for (int r = 0; r < rows; ++r)
    for (int c = 0; c < cols; ++c) {
      uint32_t u;
      std::memcpy(&u, &host[(size_t)r * cols + c], 4);
      u += 0x7fffu + ((u >> 16) & 1u);
      h[(size_t)r * ld_dev + c] = (uint16_t)(u >> 16);
    }
  hipError_t e = hipMalloc(dev, h.size() * sizeof(uint16_t));
  if (e == hipSuccess) e = hipMemcpy(*dev, h.data(), h.size() * 2, hipMemcpyHostToDevice);
  return e;
}

static hipError_t upload_f32(const float* host, int n, int n_dev, float** dev) {
  std::vector<float> h(n_dev, 0.f);
  std::memcpy(h.data(), host, sizeof(float) * n);
  hipError_t e = hipMalloc(dev, sizeof(float) * n_dev);
  if (e == hipSuccess) e = hipMemcpy(*dev, h.data(), sizeof(float) * n_dev, hipMemcpyHostToDevice);
  return e;
}

void free_mlp(cg_mlp* m) {
  if (!m) return;
  for (void* p : {(void*)m->w1, (void*)m->b1, (void*)m->w2, (void*)m->b2, (void*)m->w3,
                  (void*)m->b3})
    if (p) (void)hipFree(p);
  delete m;
}

cg_status make_mlp(const float* params, const float* mean, const float* stdv, float noise_floor,
                   cg_mlp** out) {
  cg_mlp* m = new (std::nothrow) cg_mlp();
  if (!m) return CG_ERR_OOM;
  const float* w1 = params + MLP_OFF_W1;
  const float* b1 = params + MLP_OFF_B1;
  const float* w2 = params + MLP_OFF_W2;
  const float* b2 = params + MLP_OFF_B2;
  const float* w3 = params + MLP_OFF_W3;
  const float* b3 = params + MLP_OFF_B3;
  hipError_t e = upload_bf16(w1, MLP_HID, MLP_IN, MLP_IN_PAD, &m->w1);
  if (e == hipSuccess) e = upload_f32(b1, MLP_HID, MLP_HID, &m->b1);
  if (e == hipSuccess) e = upload_bf16(w2, MLP_HID, MLP_HID, MLP_HID, &m->w2);
  if (e == hipSuccess) e = upload_f32(b2, MLP_HID, MLP_HID, &m->b2);
  if (e == hipSuccess) {
    // 4 output rows padded to one 16-row MFMA tile
    std::vector<float> w3p((size_t)16 * MLP_HID, 0.f);
    std::memcpy(w3p.data(), w3, sizeof(float) * 4 * MLP_HID);
    e = upload_bf16(w3p.data(), 16, MLP_HID, MLP_HID, &m->w3);
  }
  if (e == hipSuccess) e = upload_f32(b3, 4, 16, &m->b3);
  if (e != hipSuccess) {
    free_mlp(m);
    return hip_fail(e, "cg_set_mlp upload");
  }
  for (int j = 0; j < 4; ++j) {
    m->scale.mean[j] = mean[j];
    m->scale.std[j] = stdv[j];
  }
  m->noise_floor = noise_floor;
  *out = m;
  return CG_OK;
}

hipError_t launch_mlp_infer(const cg_mlp* m, const float* y, int64_t nf, int k, float* p0,
                            hipStream_t s, const int32_t* dev_n) {
  const int64_t blocks = (nf + IB - 1) / IB;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(mlp_infer_kernel, dim3((unsigned)blocks), dim3(256), 0, s, y, nf, k, m->w1,
                     m->b1, m->w2, m->b2, m->w3, m->b3, m->scale, p0, dev_n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// trainer

void free_trainer(cg_mlp_trainer* t) {
  if (!t) return;
  (void)hipDeviceSynchronize();
  if (t->mem) (void)hipFree(t->mem);
  delete t;
}

cg_status make_trainer(int32_t batch, const float* init, cg_mlp_trainer** out) {
  cg_mlp_trainer* t = new (std::nothrow) cg_mlp_trainer();
  if (!t) return CG_ERR_OOM;
  t->batch = batch;
  // carve one allocation
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~size_t(255);
    return o;
  };
  const size_t B = (size_t)batch;
  const size_t o_params = take(4 * MLP_NPARAMS), o_grads = take(4 * MLP_NPARAMS),
               o_m = take(4 * MLP_NPARAMS), o_v = take(4 * MLP_NPARAMS);
  const size_t o_w1b = take(2 * MLP_HID * MLP_IN), o_w2b = take(2 * MLP_HID * MLP_HID),
               o_w3b = take(2 * 4 * MLP_HID);
  const size_t o_xb = take(2 * B * MLP_IN), o_tb = take(4 * B * 4), o_wb = take(4 * B);
  const size_t o_h1 = take(4 * B * MLP_HID), o_a1b = take(2 * B * MLP_HID),
               o_h2 = take(4 * B * MLP_HID), o_a2b = take(2 * B * MLP_HID),
               o_out = take(4 * B * 4), o_dout = take(4 * B * 4), o_doutb = take(2 * B * 4),
               o_dh2 = take(4 * B * MLP_HID), o_dh2b = take(2 * B * MLP_HID),
               o_dh1 = take(4 * B * MLP_HID), o_dh1b = take(2 * B * MLP_HID),
               o_loss = take(4);
  hipError_t e = hipMalloc(&t->mem, off);
  if (e != hipSuccess) {
    delete t;
    return hip_fail(e, "trainer alloc");
  }
  char* b = static_cast<char*>(t->mem);
  t->params = reinterpret_cast<float*>(b + o_params);
  t->grads = reinterpret_cast<float*>(b + o_grads);
  t->m = reinterpret_cast<float*>(b + o_m);
  t->v = reinterpret_cast<float*>(b + o_v);
  t->w1b = reinterpret_cast<uint16_t*>(b + o_w1b);
  t->w2b = reinterpret_cast<uint16_t*>(b + o_w2b);
  t->w3b = reinterpret_cast<uint16_t*>(b + o_w3b);
  t->xb = reinterpret_cast<uint16_t*>(b + o_xb);
  t->tb = reinterpret_cast<float*>(b + o_tb);
  t->wb = reinterpret_cast<float*>(b + o_wb);
  t->h1 = reinterpret_cast<float*>(b + o_h1);
  t->a1b = reinterpret_cast<uint16_t*>(b + o_a1b);
  t->h2 = reinterpret_cast<float*>(b + o_h2);
  t->a2b = reinterpret_cast<uint16_t*>(b + o_a2b);
  t->out = reinterpret_cast<float*>(b + o_out);
  t->dout = reinterpret_cast<float*>(b + o_dout);
  t->doutb = reinterpret_cast<uint16_t*>(b + o_doutb);
  t->dh2 = reinterpret_cast<float*>(b + o_dh2);
  t->dh2b = reinterpret_cast<uint16_t*>(b + o_dh2b);
  t->dh1 = reinterpret_cast<float*>(b + o_dh1);
  t->dh1b = reinterpret_cast<uint16_t*>(b + o_dh1b);
  t->loss = reinterpret_cast<float*>(b + o_loss);
  e = hipMemcpy(t->params, init, 4 * MLP_NPARAMS, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    std::vector<float> zeros(MLP_NPARAMS, 0.f);
    e = hipMemcpy(t->m, zeros.data(), 4 * MLP_NPARAMS, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(t->v, zeros.data(), 4 * MLP_NPARAMS, hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    free_trainer(t);
    return hip_fail(e, "trainer init");
  }
  *out = t;
  return CG_OK;
}

static hipError_t refresh_bf16(cg_mlp_trainer* t, hipStream_t s) {
  auto conv = [&](const float* src, uint16_t* dst, int n) {
    hipLaunchKernelGGL(to_bf16_kernel, dim3((n + 255) / 256), dim3(256), 0, s, src, dst, n);
  };
  conv(t->params + MLP_OFF_W1, t->w1b, MLP_HID * MLP_IN);
  conv(t->params + MLP_OFF_W2, t->w2b, MLP_HID * MLP_HID);
  conv(t->params + MLP_OFF_W3, t->w3b, 4 * MLP_HID);
  return hipGetLastError();
}

// forward + loss + backward for the gathered mini-batch (xb, tb, wb) into grads
static hipError_t fwd_bwd(cg_mlp_trainer* t, hipStream_t s) {
  const int B = t->batch;
  hipError_t e = refresh_bf16(t, s);
  if (e != hipSuccess) return e;
  GemmEpi ep{};
  // forward
  ep = GemmEpi{EPI_GELU, t->params + MLP_OFF_B1, t->h1, MLP_HID, t->a1b, MLP_HID, nullptr, 0};
  if ((e = gemm<0, 0>(B, MLP_HID, MLP_IN, t->xb, MLP_IN, t->w1b, MLP_IN, ep, s)) != hipSuccess)
    return e;
  ep = GemmEpi{EPI_GELU, t->params + MLP_OFF_B2, t->h2, MLP_HID, t->a2b, MLP_HID, nullptr, 0};
  if ((e = gemm<0, 0>(B, MLP_HID, MLP_HID, t->a1b, MLP_HID, t->w2b, MLP_HID, ep, s)) != hipSuccess)
    return e;
  ep = GemmEpi{EPI_STORE, t->params + MLP_OFF_B3, t->out, 4, nullptr, 0, nullptr, 0};
  if ((e = gemm<0, 0>(B, 4, MLP_HID, t->a2b, MLP_HID, t->w3b, MLP_HID, ep, s)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(loss_kernel, dim3(1), dim3(256), 0, s, t->out, t->tb, t->wb, B, t->dout,
                     t->doutb, t->loss);
  // backward: dW3 = dOut^T A2, db3, dH2 = (dOut W3) * GELU'(H2)
  ep = GemmEpi{EPI_STORE, nullptr, t->grads + MLP_OFF_W3, MLP_HID, nullptr, 0, nullptr, 0};
  if ((e = gemm<1, 1>(4, MLP_HID, B, t->doutb, 4, t->a2b, MLP_HID, ep, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(colsum_kernel, dim3(1), dim3(64), 0, s, t->dout, B, 4, 4,
                     t->grads + MLP_OFF_B3);
  ep = GemmEpi{EPI_DGELU, nullptr, t->dh2, MLP_HID, t->dh2b, MLP_HID, t->h2, MLP_HID};
  if ((e = gemm<0, 1>(B, MLP_HID, 4, t->doutb, 4, t->w3b, MLP_HID, ep, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(colsum_kernel, dim3(1), dim3(256), 0, s, t->dh2, B, MLP_HID, MLP_HID,
                     t->grads + MLP_OFF_B2);
  ep = GemmEpi{EPI_STORE, nullptr, t->grads + MLP_OFF_W2, MLP_HID, nullptr, 0, nullptr, 0};
  if ((e = gemm<1, 1>(MLP_HID, MLP_HID, B, t->dh2b, MLP_HID, t->a1b, MLP_HID, ep, s)) != hipSuccess)
    return e;
  ep = GemmEpi{EPI_DGELU, nullptr, t->dh1, MLP_HID, t->dh1b, MLP_HID, t->h1, MLP_HID};
  if ((e = gemm<0, 1>(B, MLP_HID, MLP_HID, t->dh2b, MLP_HID, t->w2b, MLP_HID, ep, s)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(colsum_kernel, dim3(1), dim3(256), 0, s, t->dh1, B, MLP_HID, MLP_HID,
                     t->grads + MLP_OFF_B1);
  ep = GemmEpi{EPI_STORE, nullptr, t->grads + MLP_OFF_W1, MLP_IN, nullptr, 0, nullptr, 0};
  if ((e = gemm<1, 1>(MLP_HID, MLP_IN, B, t->dh1b, MLP_HID, t->xb, MLP_IN, ep, s)) != hipSuccess)
    return e;
  return hipGetLastError();
}

cg_status trainer_step(cg_mlp_trainer* t, const float* x, const float* tg, const float* w,
                       const int32_t* idx, float lr, float b1, float b2, float eps, int update,
                       float* grads_out, float* loss_out, hipStream_t s) {
  hipLaunchKernelGGL(gather_kernel, dim3(t->batch), dim3(256), 0, s, x, tg, w, idx, t->batch,
                     t->xb, t->tb, t->wb);
  hipError_t e = fwd_bwd(t, s);
  if (e != hipSuccess) return hip_fail(e, "trainer forward/backward");
  if (grads_out)
    if ((e = hipMemcpyAsync(grads_out, t->grads, 4 * MLP_NPARAMS, hipMemcpyDeviceToDevice, s)) !=
        hipSuccess)
      return hip_fail(e, "trainer grads copy");
  if (loss_out)
    if ((e = hipMemcpyAsync(loss_out, t->loss, 4, hipMemcpyDeviceToDevice, s)) != hipSuccess)
      return hip_fail(e, "trainer loss copy");
  if (update) {
    ++t->step;
    const float c1 = 1.f - (float)std::pow((double)b1, (double)t->step);
    const float c2 = 1.f - (float)std::pow((double)b2, (double)t->step);
    hipLaunchKernelGGL(adam_kernel, dim3((MLP_NPARAMS + 255) / 256), dim3(256), 0, s, t->params,
                       t->grads, t->m, t->v, MLP_NPARAMS, lr, b1, b2, eps, c1, c2);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "adam launch");
  }
  return CG_OK;
}

}  // namespace cg
