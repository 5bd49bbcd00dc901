// Real FFT of the paper's 2200-sample frames (8-bit or 16-bit samples) with
// the tooth gather, amplitude and division by the reference in the epilogue.
//
// Paper, Data Capture and Processing: the 8-bit samples are cast to single
// precision on the GPU, reshaped into rows of 2200 samples (1 us at
// 2.2 GS/s), each row is Fourier transformed and the comb-tooth bins are
// picked out and divided by the averaged reference spectrum.
//
// X[k] = sum_t x[t] e^{-2 pi i k t / 2200} through the complex FFT of the
// 1100 points z[n] = x[2n] + i x[2n+1]:
//   2 X[k] = (Z[k] + conj Z[M-k]) - i W_N^k (Z[k] - conj Z[M-k]),  M = 1100,
// evaluated only at the tooth bins.  The complex FFT is a Stockham autosort
// over the radices 4, 5, 5, 11 (1100 = 2^2 5^2 11): pass p with radix R and
// stride S (the product of the earlier radices) maps work item j (of M/R)
// through v_r = a[j + r M/R], v_r *= W_M^{(j mod S) r M/(S R)}, an R-point
// DFT, and b[(j div S) S R + (j mod S) + m S] = V_m; the odd radices use the
// pairwise form (sums and differences of v_r and v_{R-r} against cos and
// sin), about a quarter of the multiplies of the plain DFT.
//
// gfx950 layout: one wavefront per frame.  A persistent block of wavefronts
// (four, or eight in the comb shape below) shares the W_1100 table in LDS;
// each wavefront owns one 1100-
// point complex buffer in LDS and walks its own frames (stride: every
// wavefront of the grid), keeping the next frame's raw words in registers
// while the current one is transformed (non-temporal loads).  The raw words
// go to the start of the buffer as they are, and the first pass reads its
// sample pairs from there and converts them.  Each pass reads all of its
// butterfly inputs, computes them in registers and writes its outputs back to
// the same buffer; as a frame lives in one wavefront, the reads and writes
// are ordered by wavefront-scope fences instead of block barriers.  The
// twiddles come from the table; the DFT constants of the odd radices are
// literals.  Output pruning: of the last three passes only the butterflies
// whose outputs lead to a tooth bin (Z[b] or Z[M - b]) run; the plan lists
// them.  For the paper's comb (bins |51 + 10n|, all odd and = +-1 mod 10)
// that is 110 of 220, 44 of 220 and 20 of 100 butterflies.  Each lane keeps the constants of its teeth
// (bins, W_2200^bin, 0.5 / reference) in registers for the kernel's lifetime.
#include <vector>

#include "internal.h"

namespace cg {
namespace {

constexpr int MX_M = 1100;        // complex points
constexpr int MX_N = 2 * MX_M;    // samples per frame

struct cx {
  float x, y;
};

__device__ __forceinline__ cx cmul(cx a, cx b) {
  return {fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x)};
}
__device__ __forceinline__ cx cadd(cx a, cx b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cx csub(cx a, cx b) { return {a.x - b.x, a.y - b.y}; }

// A frame lives in one wavefront: its lanes run in lock step and the LDS
// executes one wavefront's accesses in issue order, so a wavefront-scope
// fence orders a pass's reads and writes against the next one's.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// cos and sin of 2 pi q / R, q = 0 .. R-1
template <int R>
struct Dft;
template <>
struct Dft<5> {
  static constexpr float C[5] = {1.000000000e+00f, 3.090169944e-01f, -8.090169944e-01f,
                                 -8.090169944e-01f, 3.090169944e-01f};
  static constexpr float S[5] = {0.000000000e+00f, 9.510565163e-01f, 5.877852523e-01f,
                                 -5.877852523e-01f, -9.510565163e-01f};
};
template <>
struct Dft<11> {
  static constexpr float C[11] = {1.000000000e+00f, 8.412535328e-01f, 4.154150130e-01f,
                                  -1.423148383e-01f, -6.548607339e-01f, -9.594929736e-01f,
                                  -9.594929736e-01f, -6.548607339e-01f, -1.423148383e-01f,
                                  4.154150130e-01f, 8.412535328e-01f};
  static constexpr float S[11] = {0.000000000e+00f, 5.406408175e-01f, 9.096319954e-01f,
                                  9.898214419e-01f, 7.557495744e-01f, 2.817325568e-01f,
                                  -2.817325568e-01f, -7.557495744e-01f, -9.898214419e-01f,
                                  -9.096319954e-01f, -5.406408175e-01f};
};

// R-point forward DFT in place.  Radix 4 directly; odd R in the pairwise form:
// with a_r = v_r + v_{R-r} and b_r = v_r - v_{R-r} (r = 1 .. (R-1)/2),
//   V_m = v_0 + sum_r a_r cos(2 pi r m / R) - i sum_r b_r sin(2 pi r m / R)
// and V_{R-m} the same with + i.
template <int R>
__device__ __forceinline__ void dft(cx (&v)[R]) {
  if constexpr (R == 4) {
    const cx s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    const cx s13 = cadd(v[1], v[3]), d13 = csub(v[1], v[3]);
    v[0] = cadd(s02, s13);
    v[2] = csub(s02, s13);
    v[1] = {d02.x + d13.y, d02.y - d13.x};  // d02 - i d13
    v[3] = {d02.x - d13.y, d02.y + d13.x};  // d02 + i d13
  } else {
    constexpr int H = (R - 1) / 2;
    cx a[H], b[H];
    cx sum = v[0];
#pragma unroll
    for (int r = 1; r <= H; ++r) {
      a[r - 1] = cadd(v[r], v[R - r]);
      b[r - 1] = csub(v[r], v[R - r]);
      sum = cadd(sum, a[r - 1]);
    }
    const cx v0 = v[0];
#pragma unroll
    for (int m = 1; m <= H; ++m) {
      cx t1 = v0, t2 = {0.f, 0.f};
#pragma unroll
      for (int r = 1; r <= H; ++r) {
        const float c = Dft<R>::C[(r * m) % R], sn = Dft<R>::S[(r * m) % R];
        t1.x = fmaf(a[r - 1].x, c, t1.x);
        t1.y = fmaf(a[r - 1].y, c, t1.y);
        t2.x = fmaf(b[r - 1].x, sn, t2.x);
        t2.y = fmaf(b[r - 1].y, sn, t2.y);
      }
      v[m] = {t1.x + t2.y, t1.y - t2.x};      // t1 - i t2
      v[R - m] = {t1.x - t2.y, t1.y + t2.x};  // t1 + i t2
    }
    v[0] = sum;
  }
}

// One Stockham pass of radix R on one frame's buffer: butterfly j (of M / R)
// takes v_r = z[j + r M/R], multiplies v_r by W_M^{(j mod S) r M/(S R)}, runs
// the R-point DFT and writes V_m to z[(j div S) S R + (j mod S) + m S].  The
// lane runs butterflies jl[q] for rounds q < nr (wave-uniform; -1: none).
// All reads precede all writes (same buffer).
template <int R, int S, int MAXR>
__device__ __forceinline__ void pass(cx* z, const cx* __restrict__ tw, const int (&jl)[MAXR],
                                     int nr) {
  constexpr int NB = MX_M / R;
  constexpr int TWS = MX_M / (S * R);
  cx v[MAXR][R];
#pragma unroll
  for (int q = 0; q < MAXR; ++q) {
    if (q < nr) {
      const int j = jl[q] < 0 ? 0 : jl[q];
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = z[j + r * NB];
      // W_M^{kk r TWS}: kk r TWS < S R TWS = M, no wrap
      const int e = (j % S) * TWS;
#pragma unroll
      for (int r = 1; r < R; ++r) v[q][r] = cmul(v[q][r], tw[e * r]);
      dft<R>(v[q]);
    }
  }
  wave_sync();
#pragma unroll
  for (int q = 0; q < MAXR; ++q) {
    const int j = jl[q];
    if (q < nr && j >= 0) {
      cx* o = z + (j / S) * S * R + j % S;
#pragma unroll
      for (int m = 0; m < R; ++m) o[m * S] = v[q][m];
    }
  }
  wave_sync();
}

// The first pass (radix 4, no twiddles) reads its complex points as sample
// pairs from the raw frame at the start of the buffer.
template <typename T>
struct Raw;
template <>
struct Raw<int8_t> {
  static constexpr int WORDS = MX_N / 4;  // 32-bit words per frame
  __device__ static cx point(const cx* z, int n) {
    const uint32_t h = reinterpret_cast<const uint16_t*>(z)[n];
    return {(float)(int8_t)(h & 0xff), (float)(int8_t)(h >> 8)};
  }
};
template <>
struct Raw<int16_t> {
  static constexpr int WORDS = MX_N / 2;
  __device__ static cx point(const cx* z, int n) {
    const int32_t w = reinterpret_cast<const int32_t*>(z)[n];
    return {(float)(int16_t)(w & 0xffff), (float)(w >> 16)};
  }
};

template <typename T>
__device__ __forceinline__ void first_pass(cx* z, int lane) {
  constexpr int R = 4, NB = MX_M / R, ROUNDS = (NB + 63) / 64;
  cx v[ROUNDS][R];
#pragma unroll
  for (int q = 0; q < ROUNDS; ++q) {
    const int j = lane + 64 * q;
    if (q < ROUNDS - 1 || j < NB) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = Raw<T>::point(z, j + r * NB);
    }
  }
#pragma unroll
  for (int q = 0; q < ROUNDS; ++q) dft<R>(v[q]);
  wave_sync();
#pragma unroll
  for (int q = 0; q < ROUNDS; ++q) {
    const int j = lane + 64 * q;
    if (q < ROUNDS - 1 || j < NB) {
      cx* o = z + j * R;
#pragma unroll
      for (int m = 0; m < R; ++m) o[m] = v[q][m];
    }
  }
  wave_sync();
}

// Launch shapes: rounds of 64 butterflies a lane may run in the last three
// passes (R1, R2, R3) and wavefronts per block.  The general shape covers any
// tooth set; the comb shape covers tooth sets whose pruned passes need at
// most 2, 1 and 1 rounds (the paper's comb): its smaller register arrays let
// four wavefronts share a SIMD, and eight-wavefront blocks share one twiddle
// table in LDS.
struct ShapeGeneral {
  static constexpr int R1 = 4, R2 = 4, R3 = 2, WAVES = 4;
};
struct ShapeComb {
  static constexpr int R1 = 2, R2 = 1, R3 = 1, WAVES = 8;
};

template <class SH>
constexpr size_t mx_lds_bytes() {
  return (size_t)(SH::WAVES + 1) * MX_M * sizeof(cx);
}

// TR = rounds of 64 teeth a lane covers (k <= 64 TR).
template <typename T, int TR, class SH>
__global__ __launch_bounds__(64 * SH::WAVES) void fft_mixed_kernel(
    const T* __restrict__ frames, int64_t n_frames, const int32_t* __restrict__ bins,
    const float* __restrict__ half_inv_ref, const cx* __restrict__ tw_m,
    const cx* __restrict__ tw_tooth, int k, const int16_t* __restrict__ lists, int nr1, int nr2,
    int nr3, float* __restrict__ out_mag, float* __restrict__ out_y,
    const int32_t* __restrict__ dev_n) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  cx* tw = reinterpret_cast<cx*>(lds);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  cx* z = tw + MX_M * (1 + wv);
  if (dev_n) {
    const int64_t dn = *dev_n;
    n_frames = dn < n_frames ? dn : n_frames;
  }
  constexpr int WAVES = SH::WAVES;
  if ((int64_t)blockIdx.x * WAVES >= n_frames) return;  // uniform over the block
  for (int e = threadIdx.x; e < MX_M; e += 64 * WAVES) tw[e] = tw_m[e];
  // this lane's teeth: i = lane + 64 q
  int lo[TR], hi[TR];
  cx tt[TR];
  float thr[TR];
#pragma unroll
  for (int q = 0; q < TR; ++q) {
    const int i = lane + 64 * q;
    const int b = i < k ? bins[i] : 0;
    lo[q] = b % MX_M;
    hi[q] = (MX_M - b) % MX_M;
    tt[q] = i < k ? tw_tooth[i] : cx{0.f, 0.f};
    thr[q] = i < k ? half_inv_ref[i] : 0.f;
  }
  // this lane's butterflies in the last three passes
  int j1[SH::R1], j2[SH::R2], j3[SH::R3];
#pragma unroll
  for (int q = 0; q < SH::R1; ++q) j1[q] = q < nr1 ? lists[64 * q + lane] : -1;
#pragma unroll
  for (int q = 0; q < SH::R2; ++q) j2[q] = q < nr2 ? lists[64 * (nr1 + q) + lane] : -1;
#pragma unroll
  for (int q = 0; q < SH::R3; ++q) j3[q] = q < nr3 ? lists[64 * (nr1 + nr2 + q) + lane] : -1;
  __syncthreads();  // the twiddle table; no block barrier after this
  using RW = Raw<T>;
  constexpr int WPL = (RW::WORDS + 63) / 64;  // raw words per lane
  const int32_t* words = reinterpret_cast<const int32_t*>(frames);
  const int64_t stride = (int64_t)gridDim.x * WAVES;
  int64_t f = (int64_t)blockIdx.x * WAVES + wv;
  int32_t raw[WPL];
  auto fetch = [&](int64_t fr) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < WPL; ++u) {
      const int w = lane + 64 * u;
      raw[u] = (u < WPL - 1 || w < RW::WORDS)
                   ? __builtin_nontemporal_load(words + fr * RW::WORDS + w)
                   : 0;
    }
  };
  if (f < n_frames) fetch(f);
  for (; f < n_frames; f += stride) {
    int32_t* zw = reinterpret_cast<int32_t*>(z);
#pragma unroll
    for (int u = 0; u < WPL; ++u) {
      const int w = lane + 64 * u;
      if (u < WPL - 1 || w < RW::WORDS) zw[w] = raw[u];
    }
    if (f + stride < n_frames) fetch(f + stride);  // next frame in flight
    wave_sync();
    first_pass<T>(z, lane);
    pass<5, 4, SH::R1>(z, tw, j1, nr1);
    pass<5, 20, SH::R2>(z, tw, j2, nr2);
    pass<11, 100, SH::R3>(z, tw, j3, nr3);
    // epilogue: 2 X[b] = (Z[b] + conj Z[M-b]) - i W_N^b (Z[b] - conj Z[M-b])
#pragma unroll
    for (int q = 0; q < TR; ++q) {
      const int i = lane + 64 * q;
      if (i < k) {
        const cx za = z[lo[q]];
        const cx zb = z[hi[q]];                   // conj taken below
        const cx sm = {za.x + zb.x, za.y - zb.y};  // Z[b] + conj Z[M-b]
        const cx df = {za.x - zb.x, za.y + zb.y};  // Z[b] - conj Z[M-b]
        const cx wd = cmul(tt[q], df);
        const float re = sm.x + wd.y, im = sm.y - wd.x;  // sm - i W df
        const float two_mag = sqrtf(fmaf(re, re, im * im));
        const int64_t o = f * k + i;
        if (out_mag) out_mag[o] = 0.5f * two_mag;
        if (out_y) out_y[o] = two_mag * thr[q];
      }
    }
    wave_sync();  // the epilogue's reads before the next frame's raw words
  }
}

template <typename T, int TR, class SH>
int mx_grid_limit_t(const cg_plan* p) {
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fft_mixed_kernel<T, TR, SH>,
                                                   64 * SH::WAVES,
                                                   mx_lds_bytes<SH>()) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) !=
          hipSuccess ||
      per_cu <= 0 || cus <= 0)
    return 0;
  return per_cu * cus;
}

template <typename T, int TR, class SH>
hipError_t launch_mx_t(const cg_plan* p, const void* frames, int64_t nf, float* out_mag,
                       float* out_y, hipStream_t s, const int32_t* dev_n) {
  int64_t blocks = (nf + SH::WAVES - 1) / SH::WAVES;
  if (p->fft_blocks > 0 && blocks > p->fft_blocks) blocks = p->fft_blocks;
  if (p->fft_cap > 0 && blocks > p->fft_cap) blocks = p->fft_cap;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  if (blocks == 0) return hipSuccess;
  fft_mixed_kernel<T, TR, SH><<<dim3((unsigned)blocks), dim3(64 * SH::WAVES),
                                mx_lds_bytes<SH>(), s>>>(
      static_cast<const T*>(frames), nf, p->d_bins, p->d_half_inv_ref,
      reinterpret_cast<const cx*>(p->d_tw_mixed), reinterpret_cast<const cx*>(p->d_tooth_w),
      p->k, p->d_mx_list, p->mx_rounds[0], p->mx_rounds[1], p->mx_rounds[2], out_mag, out_y,
      dev_n);
  return hipGetLastError();
}

// The comb shape when the plan's pruned passes fit it.
bool comb_shape(const cg_plan* p) {
  return p->mx_rounds[0] <= ShapeComb::R1 && p->mx_rounds[1] <= ShapeComb::R2 &&
         p->mx_rounds[2] <= ShapeComb::R3;
}

// One instantiation per tooth rounds (k <= CG_MAX_TEETH = 440: up to 7) and
// launch shape.
template <typename T, class SH>
int mx_grid_limit_s(const cg_plan* p) {
  switch ((p->k + 63) / 64) {
    case 1: return mx_grid_limit_t<T, 1, SH>(p);
    case 2: return mx_grid_limit_t<T, 2, SH>(p);
    case 3: return mx_grid_limit_t<T, 3, SH>(p);
    case 4: return mx_grid_limit_t<T, 4, SH>(p);
    case 5: return mx_grid_limit_t<T, 5, SH>(p);
    case 6: return mx_grid_limit_t<T, 6, SH>(p);
    case 7: return mx_grid_limit_t<T, 7, SH>(p);
    default: return 0;
  }
}

template <typename T>
int mx_grid_limit(const cg_plan* p) {
  return comb_shape(p) ? mx_grid_limit_s<T, ShapeComb>(p) : mx_grid_limit_s<T, ShapeGeneral>(p);
}

template <typename T, class SH>
hipError_t launch_mx_s(const cg_plan* p, const void* frames, int64_t nf, float* out_mag,
                       float* out_y, hipStream_t s, const int32_t* dev_n) {
  switch ((p->k + 63) / 64) {
    case 1: return launch_mx_t<T, 1, SH>(p, frames, nf, out_mag, out_y, s, dev_n);
    case 2: return launch_mx_t<T, 2, SH>(p, frames, nf, out_mag, out_y, s, dev_n);
    case 3: return launch_mx_t<T, 3, SH>(p, frames, nf, out_mag, out_y, s, dev_n);
    case 4: return launch_mx_t<T, 4, SH>(p, frames, nf, out_mag, out_y, s, dev_n);
    case 5: return launch_mx_t<T, 5, SH>(p, frames, nf, out_mag, out_y, s, dev_n);
    case 6: return launch_mx_t<T, 6, SH>(p, frames, nf, out_mag, out_y, s, dev_n);
    case 7: return launch_mx_t<T, 7, SH>(p, frames, nf, out_mag, out_y, s, dev_n);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_mx(const cg_plan* p, const void* frames, int64_t nf, float* out_mag,
                     float* out_y, hipStream_t s, const int32_t* dev_n) {
  return comb_shape(p) ? launch_mx_s<T, ShapeComb>(p, frames, nf, out_mag, out_y, s, dev_n)
                       : launch_mx_s<T, ShapeGeneral>(p, frames, nf, out_mag, out_y, s, dev_n);
}

}  // namespace

hipError_t mixed_prepare(cg_plan* p) {
  // Backwards from the needed outputs of the last pass: a butterfly is needed
  // when one of its outputs is, and then all of its inputs are.
  constexpr int RAD[3] = {5, 5, 11}, STR[3] = {4, 20, 100};
  std::vector<char> need(MX_M, 0);
  for (int32_t b : p->h_bins) {
    need[b % MX_M] = 1;
    need[(MX_M - b) % MX_M] = 1;
  }
  std::vector<int> js[3];
  for (int ps = 2; ps >= 0; --ps) {
    const int R = RAD[ps], S = STR[ps], NB = MX_M / R;
    std::vector<char> prev(MX_M, 0);
    for (int j = 0; j < NB; ++j) {
      bool any = false;
      for (int m = 0; m < R; ++m) any = any || need[(j / S) * S * R + j % S + m * S];
      if (!any) continue;
      js[ps].push_back(j);
      for (int r = 0; r < R; ++r) prev[j + r * NB] = 1;
    }
    need.swap(prev);
  }
  std::vector<int16_t> all;
  for (int ps = 0; ps < 3; ++ps) {
    const int rounds = ((int)js[ps].size() + 63) / 64;
    p->mx_rounds[ps] = rounds;
    for (int e = 0; e < 64 * rounds; ++e)
      all.push_back(e < (int)js[ps].size() ? (int16_t)js[ps][e] : (int16_t)-1);
  }
  hipError_t e = hipMalloc(&p->d_mx_list, all.size() * sizeof(int16_t));
  if (e != hipSuccess) return e;
  return hipMemcpy(p->d_mx_list, all.data(), all.size() * sizeof(int16_t), hipMemcpyHostToDevice);
}

int fft_mixed_grid_limit(const cg_plan* p) {
  return p->sample_bytes == 1 ? mx_grid_limit<int8_t>(p) : mx_grid_limit<int16_t>(p);
}

hipError_t launch_fft_mixed(const cg_plan* p, const void* frames, int64_t nf, float* out_mag,
                            float* out_y, hipStream_t s, const int32_t* dev_n) {
  if (p->n != MX_N) return hipErrorInvalidValue;
  return p->sample_bytes == 1 ? launch_mx<int8_t>(p, frames, nf, out_mag, out_y, s, dev_n)
                              : launch_mx<int16_t>(p, frames, nf, out_mag, out_y, s, dev_n);
}

}  // namespace cg
