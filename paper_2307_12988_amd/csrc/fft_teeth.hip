// Ingest + real FFT + tooth gather + amplitude + division by the reference.
//
// Paper, Data Capture and Processing: integer samples are cast to single
// precision on the GPU, reshaped into one frame per row, every row is Fourier
// transformed, the bins of the comb teeth are selected in optical order and
// divided by the averaged reference spectrum.
//
// gfx950 design
// -------------
// * A real frame of N samples is read as N/2 complex points z[t] = x[2t] +
//   i x[2t+1] (one 32-bit load carries both int16 samples), transformed by a
//   complex FFT of M = N/2 points, and the tooth bins are untangled from Z:
//     X[k] = (Z[k] + conj Z[M-k]) / 2 - i W_N^k (Z[k] - conj Z[M-k]) / 2.
//   Only the K tooth bins are untangled; the full spectrum never leaves LDS.
// * Stockham autosort passes, 16 points per thread held in registers: two
//   radix-16 passes and one radix-M/256 pass (M = 256 .. 4096).  Threads per
//   frame T = M/16; a 256-thread workgroup holds 256/T frames.  LDS holds
//   interleaved complex points (one 64-bit access per point) with one padding
//   point per 16 so the strided pass-1 stores are bank-conflict free.
// * When a frame spans 2 or 4 rows of one wavefront (M = 512, 1024) the last
//   pass needs no LDS: its butterfly inputs sit in one register of the
//   frame's rows, and the lane swaps of gfx950 (permlane16/32 swap) transpose
//   them into one lane.  A frame then goes through LDS once between passes
//   1 and 2 and once more for the tooth gather; larger frames span several
//   wavefronts and exchange through LDS before every pass.
// * Twiddles come from a table of W_N^e built on the host in FP64 and rounded
//   once to FP32 (no fast-math sin/cos on the device).
// * Persistent blocks: the grid is sized to what fits on the chip, each block
//   walks frame groups and prefetches the next group's samples into registers
//   while it transforms the current one.  A partially filled last group masks
//   its loads and stores but keeps every barrier.
#include "internal.h"

namespace cg {
namespace {

struct __attribute__((aligned(8))) c32 {
  float x, y;
};

__device__ __forceinline__ c32 cadd(c32 a, c32 b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ c32 csub(c32 a, c32 b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ c32 cmul(c32 a, c32 b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ __forceinline__ c32 mul_mi(c32 a) { return {a.y, -a.x}; }  // -i a

constexpr float kC1 = 0.92387953251128674f;  // cos(pi/8)
constexpr float kS1 = 0.38268343236508977f;  // sin(pi/8)
constexpr float kC2 = 0.70710678118654752f;  // cos(pi/4)

// Forward DFTs of length 2, 4, 8, 16 in registers; results in natural order.
__device__ __forceinline__ void dft2(c32& a, c32& b) {
  c32 t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

__device__ __forceinline__ void dft4(c32& a0, c32& a1, c32& a2, c32& a3) {
  c32 s02 = cadd(a0, a2), d02 = csub(a0, a2);
  c32 s13 = cadd(a1, a3), d13 = mul_mi(csub(a1, a3));
  a0 = cadd(s02, s13);
  a2 = csub(s02, s13);
  a1 = cadd(d02, d13);
  a3 = csub(d02, d13);
}

__device__ __forceinline__ c32 w8_1(c32 a) { return {kC2 * (a.x + a.y), kC2 * (a.y - a.x)}; }
__device__ __forceinline__ c32 w8_3(c32 a) { return {kC2 * (a.y - a.x), -kC2 * (a.x + a.y)}; }

__device__ __forceinline__ void dft8(c32* v) {
  // n = 2 n1 + n2: DFT4 over n1, twiddle W8^(n2 k1), DFT2 over n2.
  dft4(v[0], v[2], v[4], v[6]);
  dft4(v[1], v[3], v[5], v[7]);
  v[3] = w8_1(v[3]);
  v[5] = mul_mi(v[5]);
  v[7] = w8_3(v[7]);
  dft2(v[0], v[1]);
  dft2(v[2], v[3]);
  dft2(v[4], v[5]);
  dft2(v[6], v[7]);
  // X[k1] in v[2 k1], X[k1 + 4] in v[2 k1 + 1]
  c32 t[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) t[i] = v[i];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    v[k1] = t[2 * k1];
    v[k1 + 4] = t[2 * k1 + 1];
  }
}

__device__ __forceinline__ void dft16(c32* v) {
  // n = 4 n1 + n2: DFT4 over n1 for each n2, twiddle W16^(n2 k1), DFT4 over n2.
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) dft4(v[n2], v[4 + n2], v[8 + n2], v[12 + n2]);
  // v[4 k1 + n2] holds Y[n2][k1]
  const c32 w1 = {kC1, -kS1}, w3 = {kS1, -kC1}, w9 = {-kC1, kS1};
  v[5] = cmul(v[5], w1);                       // k1=1 n2=1 : W^1
  v[6] = {kC2 * (v[6].x + v[6].y), kC2 * (v[6].y - v[6].x)};    // k1=1 n2=2 : W^2
  v[7] = cmul(v[7], w3);                       // k1=1 n2=3 : W^3
  v[9] = {kC2 * (v[9].x + v[9].y), kC2 * (v[9].y - v[9].x)};    // k1=2 n2=1 : W^2
  v[10] = mul_mi(v[10]);                       // k1=2 n2=2 : W^4
  v[11] = {kC2 * (v[11].y - v[11].x), -kC2 * (v[11].x + v[11].y)};  // k1=2 n2=3 : W^6
  v[13] = cmul(v[13], w3);                     // k1=3 n2=1 : W^3
  v[14] = {kC2 * (v[14].y - v[14].x), -kC2 * (v[14].x + v[14].y)};  // k1=3 n2=2 : W^6
  v[15] = cmul(v[15], w9);                     // k1=3 n2=3 : W^9
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) dft4(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
  // X[k1 + 4 k2] in v[4 k1 + k2]: transpose the 4x4 block
  c32 t[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) t[i] = v[i];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = t[4 * k1 + k2];
}

template <int R>
__device__ __forceinline__ void dft_r(c32* v) {
  if constexpr (R == 2) {
    dft2(v[0], v[1]);
  } else if constexpr (R == 4) {
    dft4(v[0], v[1], v[2], v[3]);
  } else if constexpr (R == 8) {
    dft8(v);
  } else {
    dft16(v);
  }
}

__device__ __forceinline__ int padx(int i) { return i + (i >> 4); }

// a * W_16^e for a compile-time e (after unrolling): quarter turns are sign
// and swap changes, eighth turns two adds and two multiplies.
__device__ __forceinline__ c32 mul_w16(c32 a, int e) {
  e &= 15;
  switch (e) {
    case 0: return a;
    case 4: return mul_mi(a);
    case 8: return {-a.x, -a.y};
    case 12: return {-a.y, a.x};
    case 2: return {kC2 * (a.x + a.y), kC2 * (a.y - a.x)};
    case 6: return {kC2 * (a.y - a.x), -kC2 * (a.x + a.y)};
    case 10: return {-kC2 * (a.x + a.y), kC2 * (a.x - a.y)};
    case 14: return {kC2 * (a.x - a.y), kC2 * (a.x + a.y)};
    default: {
      // W_16^e = cos(2 pi e / 16) - i sin(2 pi e / 16), odd e
      constexpr float c[8] = {kC1, kS1, -kS1, -kC1, -kC1, -kS1, kS1, kC1};
      constexpr float sn[8] = {kS1, kC1, kC1, kS1, -kS1, -kC1, -kC1, -kS1};
      const int h = e >> 1;
      return cmul(a, c32{c[h], -sn[h]});
    }
  }
}



// Lane exchanges of gfx950 (one row = 16 lanes of a wavefront).  swap32
// trades lanes 32..63 of a with lanes 0..31 of b; swap16 trades rows 1 and 3
// of a with rows 0 and 2 of b.
__device__ __forceinline__ float2 swap_pair32(float a, float b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                  false);
  return {__uint_as_float(r[0]), __uint_as_float(r[1])};
}
__device__ __forceinline__ float2 swap_pair16(float a, float b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                  false);
  return {__uint_as_float(r[0]), __uint_as_float(r[1])};
}
__device__ __forceinline__ void swap32(c32& a, c32& b) {
  const float2 x = swap_pair32(a.x, b.x), y = swap_pair32(a.y, b.y);
  a = {x.x, y.x};
  b = {x.y, y.y};
}
__device__ __forceinline__ void swap16(c32& a, c32& b) {
  const float2 x = swap_pair16(a.x, b.x), y = swap_pair16(a.y, b.y);
  a = {x.x, y.x};
  b = {x.y, y.y};
}

// Transpose R registers against the R rows of a frame (R = 2 or 4): on
// return, register t of row s holds what register s of row t held.
template <int R>
__device__ __forceinline__ void rows_transpose(c32* x) {
  if constexpr (R == 4) {
    swap32(x[0], x[2]);
    swap32(x[1], x[3]);
  }
  swap16(x[0], x[1]);
  if constexpr (R == 4) swap16(x[2], x[3]);
}

// Ordering of the LDS exchanges between passes.  With T <= 64 every frame
// lives inside one wavefront: its lanes run in lock step and the LDS executes
// one wavefront's accesses in issue order, so a compiler-level fence at
// wavefront scope is all a pass needs before reading what the previous pass
// wrote.  Larger frames span several wavefronts and take a block barrier.
template <int T>
__device__ __forceinline__ void frame_sync() {
  if constexpr (T <= 64) {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  } else {
    __syncthreads();
  }
}

template <int LOGM>
struct FftShape {
  static constexpr int M = 1 << LOGM;
  static constexpr int T = M / 16;          // threads per frame
  static constexpr int FPB = 256 / T;       // frames per 256-thread block
  static constexpr int PM = M + M / 16;     // padded plane length
  static constexpr int R3 = M / 256;        // radix of the last pass (1 = none)
  static constexpr int NB3 = R3 > 1 ? 16 / R3 : 0;  // last-pass butterflies per thread
  // the last pass by lane exchanges: a frame of 2 or 4 rows in one wavefront
  static constexpr bool LANE_PASS3 = R3 == 2 || R3 == 4;
  // LDS position of spectrum bin k.  The lane pass stores the spectrum with
  // consecutive lanes on consecutive bins, so it needs no padding, and an
  // evenly spaced comb with an odd spacing then gathers from distinct banks;
  // the LDS passes leave it in the padded layout.
  static __device__ __forceinline__ int fpos(int k) { return LANE_PASS3 ? k : k + (k >> 4); }
  static constexpr size_t PLANE_BYTES = sizeof(float) * 2 * FPB * PM;  // complex points
};

// Tooth constants: one float4 per tooth in LDS, {LDS positions of Z[k] and
// Z[M-k] packed in two 16-bit fields, Re W_N^k, Im W_N^k, 0.5 / ref}.  With
// TPT > 0 thread j of a frame handles the teeth j + T u, u < TPT, and also
// keeps their gather addresses in registers, so a frame's gathers and constant
// reads are issued together (one LDS round trip); TPT = 0 (more than 4 teeth
// per thread) walks the table.
template <int LOGM>
int fft_teeth_per_thread(int k) {
  const int per = (k + FftShape<LOGM>::T - 1) / FftShape<LOGM>::T;
  return per <= 1 ? 1 : per <= 2 ? 2 : per <= 4 ? 4 : 0;
}

// Dynamic LDS: the complex points of FPB frames, then the tooth table.
template <int LOGM>
size_t fft_lds_bytes(int k) {
  return FftShape<LOGM>::PLANE_BYTES + sizeof(float4) * (size_t)k;
}

// Persistent form: the grid holds as many blocks as fit on the chip and each
// block walks frame groups g = blockIdx.x, g + gridDim.x, ...  While a group
// is transformed, the 64 bytes per thread of the next group are already in
// flight (issued right after the current group's samples are converted), so
// HBM sees a steady stream of loads instead of one burst per block.  Nothing
// else is read from global memory inside the loop: twiddles and tooth
// constants live in registers (or LDS), so waiting for one load never means
// waiting for the prefetch.
template <int LOGM, int TPT>
__global__ __launch_bounds__(256) void fft_teeth_kernel(
    const int32_t* __restrict__ frames, int64_t n_frames, const int32_t* __restrict__ bins,
    const float* __restrict__ half_inv_ref, const c32* __restrict__ tw, int k_teeth,
    float* __restrict__ out_mag, float* __restrict__ out_y, const int32_t* __restrict__ dev_n) {
  using S = FftShape<LOGM>;
  constexpr int M = S::M, T = S::T, FPB = S::FPB, PM = S::PM, R3 = S::R3, NB3 = S::NB3;
  constexpr int N = 2 * M;
  extern __shared__ float4 lds4[];
  c32* s_c = reinterpret_cast<c32*>(lds4);  // FPB frames x PM complex points
  float4* s_tooth = reinterpret_cast<float4*>(s_c + FPB * PM);

  if (dev_n) {
    const int64_t dn = *dev_n;
    n_frames = dn < n_frames ? dn : n_frames;
  }
  const int64_t ngroups = (n_frames + FPB - 1) / FPB;
  int64_t g = blockIdx.x;
  if (g >= ngroups) return;  // uniform over the block

  const int tid = threadIdx.x;
  const int fl = tid / T;
  const int j = tid - fl * T;
  c32* zc = s_c + fl * PM;

  // per-tooth constants
  auto tooth_const = [&](int i) {
    const int kb = bins[i];
    const int ia = kb & (M - 1);
    const int ib = (M - kb) & (M - 1);
    const uint32_t packed = (uint32_t)S::fpos(ia) | ((uint32_t)S::fpos(ib) << 16);
    const c32 w = tw[kb];
    return make_float4(__uint_as_float(packed), w.x, w.y, half_inv_ref[i]);
  };
  for (int i = tid; i < k_teeth; i += 256) s_tooth[i] = tooth_const(i);
  // TPT > 0: LDS addresses of Z[k] and Z[M-k] in this frame's plane for the
  // teeth j + T u; teeth past the end repeat the last one (their results are
  // not stored)
  const char* t_za[TPT > 0 ? TPT : 1];
  const char* t_zb[TPT > 0 ? TPT : 1];
  if constexpr (TPT > 0) {
#pragma unroll
    for (int u = 0; u < TPT; ++u) {
      const int i = j + T * u;
      const uint32_t packed = __float_as_uint(tooth_const(i < k_teeth ? i : k_teeth - 1).x);
      t_za[u] = reinterpret_cast<const char*>(zc + (packed & 0xffffu));
      t_zb[u] = reinterpret_cast<const char*>(zc + (packed >> 16));
    }
  }
  // twiddles of pass 2 (W_256^(jm r) = W_N^(e2 r)) and pass 3 (W_M^(jp r))
  const int jm = j & 15;
  const int e2 = jm * (N / 256);
  c32 w2[15];
#pragma unroll
  for (int r = 1; r < 16; ++r) w2[r - 1] = tw[e2 * r];
  // Pass 3 twiddles W_M^((j + T q) r) = W_M^(j r) W_16^(q r): only the first
  // factor is kept per thread, the second is a compile-time constant.
  c32 w3[R3 > 1 ? R3 - 1 : 1];
  if constexpr (R3 > 1) {
#pragma unroll
    for (int r = 1; r < R3; ++r) w3[r - 1] = tw[2 * j * r];
  }

  // first group's samples.  Threads of frames past the end read the last
  // frame instead (their results are never stored), so every load is
  // unconditional.
  const int64_t last = n_frames - 1;
  int32_t raw[16];
  {
    int64_t frame = g * FPB + fl;
    frame = frame < last ? frame : last;
    const int32_t* src = frames + frame * M + j;
#pragma unroll
    for (int r = 0; r < 16; ++r) raw[r] = __builtin_nontemporal_load(src + r * T);
  }

  __syncthreads();  // the per-tooth table is filled by the whole block

  for (; g < ngroups; g += gridDim.x) {
    const int64_t frame = g * FPB + fl;
    const bool live = frame < n_frames;
    c32 v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      v[r].x = (float)(int16_t)(raw[r] & 0xffff);
      v[r].y = (float)(raw[r] >> 16);
    }
    // prefetch the next group of this block
    {
      int64_t fn = (g + gridDim.x) * FPB + fl;
      fn = fn < last ? fn : last;
      const int32_t* src = frames + fn * M + j;
#pragma unroll
      for (int r = 0; r < 16; ++r) raw[r] = __builtin_nontemporal_load(src + r * T);
    }

    // ---- pass 1: radix 16, Ns = 1 ----
    dft16(v);
    frame_sync<T>();  // the previous group's epilogue has read the points
    {
      c32* w = zc + 17 * j;  // padx(16 j + r) = 17 j + r
#pragma unroll
      for (int r = 0; r < 16; ++r) w[r] = v[r];
    }
    frame_sync<T>();
    // ---- pass 2: radix 16, Ns = 16 ----
    {
      constexpr int S2 = T + T / 16;
      const c32* rd = zc + j + (j >> 4);
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] = rd[r * S2];
      frame_sync<T>();
#pragma unroll
      for (int r = 1; r < 16; ++r) v[r] = cmul(v[r], w2[r - 1]);
      dft16(v);
      if constexpr (!S::LANE_PASS3) {
        const int base = (j >> 4) * 256 + jm;
        c32* w = zc + base + (base >> 4);
#pragma unroll
        for (int r = 0; r < 16; ++r) w[17 * r] = v[r];
      }
    }
    if constexpr (!S::LANE_PASS3) frame_sync<T>();
    // ---- pass 3: radix M/256, Ns = 256 ----
    if constexpr (S::LANE_PASS3) {
      // Register r of row s now holds point 256 s + jm + 16 r, so the R3
      // inputs of a butterfly sit in one register of the frame's R3 rows.
      // A transpose of each run of R3 registers against the rows hands row
      // s the butterfly of register q R3 + s: point j + T q and its
      // partners, the same butterflies and twiddles as the LDS form below.
#pragma unroll
      for (int q = 0; q < NB3; ++q) {
        rows_transpose<R3>(v + q * R3);
#pragma unroll
        for (int r = 1; r < R3; ++r) v[q * R3 + r] = mul_w16(cmul(v[q * R3 + r], w3[r - 1]), q * r);
        dft_r<R3>(v + q * R3);
      }
      frame_sync<T>();  // pass 2 has read the points
#pragma unroll
      for (int q = 0; q < NB3; ++q) {
        c32* w = zc + j + T * q;
#pragma unroll
        for (int r = 0; r < R3; ++r) w[256 * r] = v[q * R3 + r];
      }
      frame_sync<T>();
    } else if constexpr (R3 > 1) {
#pragma unroll
      for (int q = 0; q < NB3; ++q) {
        const int jp = j + T * q;
        const c32* rd = zc + jp + (jp >> 4);
#pragma unroll
        for (int r = 0; r < R3; ++r) v[q * R3 + r] = rd[272 * r];
      }
      frame_sync<T>();
#pragma unroll
      for (int q = 0; q < NB3; ++q) {
        const int jp = j + T * q;
#pragma unroll
        for (int r = 1; r < R3; ++r) v[q * R3 + r] = mul_w16(cmul(v[q * R3 + r], w3[r - 1]), q * r);
        dft_r<R3>(v + q * R3);
        c32* w = zc + jp + (jp >> 4);
#pragma unroll
        for (int r = 0; r < R3; ++r) w[272 * r] = v[q * R3 + r];
      }
      frame_sync<T>();
    }
    // ---- untangle the real spectrum at the tooth bins, amplitude, / ref ----
    const int64_t row = frame * k_teeth;
    auto tooth_out = [&](const float4 t, c32 a, c32 zb, int i) {
      const c32 b = {zb.x, -zb.y};  // conj Z[M-k]
      const c32 sm = cadd(a, b);
      const c32 o = mul_mi(csub(a, b));
      const c32 x = cadd(sm, cmul(c32{t.y, t.z}, o));
      const float r2 = __builtin_amdgcn_sqrtf(x.x * x.x + x.y * x.y);  // 2 |X[k]|
      if (out_mag) out_mag[row + i] = 0.5f * r2;
      if (out_y) out_y[row + i] = r2 * t.w;
    };
    if constexpr (TPT > 0) {
      // all gathers of the frame at once, one LDS round trip
      c32 za[TPT], zb[TPT];
      float4 tc[TPT];
#pragma unroll
      for (int u = 0; u < TPT; ++u) {
        const int i = j + T * u;
        tc[u] = s_tooth[i < k_teeth ? i : k_teeth - 1];
        za[u] = *reinterpret_cast<const c32*>(t_za[u]);
        zb[u] = *reinterpret_cast<const c32*>(t_zb[u]);
      }
      if (live) {
#pragma unroll
        for (int u = 0; u < TPT; ++u)
          if (j + T * u < k_teeth) tooth_out(tc[u], za[u], zb[u], j + T * u);
      }
    } else if (live) {
      for (int i = j; i < k_teeth; i += T) {
        const float4 t = s_tooth[i];
        const uint32_t packed = __float_as_uint(t.x);
        tooth_out(t, zc[packed & 0xffffu], zc[packed >> 16], i);
      }
    }
  }
}

template <int LOGM, int TPT>
int max_blocks_tt(const cg_plan* p) {
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fft_teeth_kernel<LOGM, TPT>, 256,
                                                   fft_lds_bytes<LOGM>(p->k)) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) !=
          hipSuccess ||
      per_cu <= 0 || cus <= 0)
    return 0;
  return per_cu * cus;
}

template <int LOGM>
int max_blocks_t(const cg_plan* p) {
  switch (fft_teeth_per_thread<LOGM>(p->k)) {
    case 1: return max_blocks_tt<LOGM, 1>(p);
    case 2: return max_blocks_tt<LOGM, 2>(p);
    case 4: return max_blocks_tt<LOGM, 4>(p);
    default: return max_blocks_tt<LOGM, 0>(p);
  }
}

template <int LOGM, int TPT>
hipError_t launch_tt(const cg_plan* p, const void* frames, int64_t nf, float* out_mag,
                     float* out_y, hipStream_t s, const int32_t* dev_n) {
  using S = FftShape<LOGM>;
  int64_t blocks = (nf + S::FPB - 1) / S::FPB;
  if (p->fft_blocks > 0 && blocks > p->fft_blocks) blocks = p->fft_blocks;
  if (p->fft_cap > 0 && blocks > p->fft_cap) blocks = p->fft_cap;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  if (blocks == 0) return hipSuccess;
  fft_teeth_kernel<LOGM, TPT><<<dim3((unsigned)blocks), dim3(256), fft_lds_bytes<LOGM>(p->k),
                                 s>>>(reinterpret_cast<const int32_t*>(frames), nf, p->d_bins,
                                      p->d_half_inv_ref, reinterpret_cast<const c32*>(p->d_tw),
                                      p->k, out_mag, out_y, dev_n);
  return hipGetLastError();
}

template <int LOGM>
hipError_t launch_t(const cg_plan* p, const void* frames, int64_t nf, float* out_mag,
                    float* out_y, hipStream_t s, const int32_t* dev_n) {
  switch (fft_teeth_per_thread<LOGM>(p->k)) {
    case 1: return launch_tt<LOGM, 1>(p, frames, nf, out_mag, out_y, s, dev_n);
    case 2: return launch_tt<LOGM, 2>(p, frames, nf, out_mag, out_y, s, dev_n);
    case 4: return launch_tt<LOGM, 4>(p, frames, nf, out_mag, out_y, s, dev_n);
    default: return launch_tt<LOGM, 0>(p, frames, nf, out_mag, out_y, s, dev_n);
  }
}

}  // namespace

int fft_grid_limit(const cg_plan* p) {
  if (p->n == 2200) return fft_mixed_grid_limit(p);
  switch (p->m) {
    case 256: return max_blocks_t<8>(p);
    case 512: return max_blocks_t<9>(p);
    case 1024: return max_blocks_t<10>(p);
    case 2048: return max_blocks_t<11>(p);
    case 4096: return max_blocks_t<12>(p);
    default: return 0;
  }
}

hipError_t launch_fft_teeth(const cg_plan* p, const void* frames, int64_t nf, float* out_mag,
                            float* out_y, hipStream_t s, const int32_t* dev_n) {
  if (p->n == 2200) return launch_fft_mixed(p, frames, nf, out_mag, out_y, s, dev_n);
  if (p->sample_bytes != 2) return hipErrorInvalidValue;
  switch (p->m) {
    case 256: return launch_t<8>(p, frames, nf, out_mag, out_y, s, dev_n);
    case 512: return launch_t<9>(p, frames, nf, out_mag, out_y, s, dev_n);
    case 1024: return launch_t<10>(p, frames, nf, out_mag, out_y, s, dev_n);
    case 2048: return launch_t<11>(p, frames, nf, out_mag, out_y, s, dev_n);
    case 4096: return launch_t<12>(p, frames, nf, out_mag, out_y, s, dev_n);
    default: return hipErrorInvalidValue;
  }
}

namespace {

__global__ __launch_bounds__(256) void column_mean_kernel(const float* __restrict__ mags,
                                                          int64_t n, int k,
                                                          float* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k) return;
  double acc = 0.0;
  for (int64_t f = 0; f < n; ++f) acc += (double)mags[f * k + i];
  out[i] = (float)(acc / (double)n);
}

}  // namespace

hipError_t launch_column_mean(const float* mags, int64_t n, int k, float* out, hipStream_t s) {
  hipLaunchKernelGGL(column_mean_kernel, dim3((k + 255) / 256), dim3(256), 0, s, mags, n, k, out);
  return hipGetLastError();
}

}  // namespace cg
