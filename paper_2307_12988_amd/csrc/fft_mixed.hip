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
// gfx950 layout: a persistent block of 256 threads takes 2 frames at a time
// into LDS (two ping-pong buffers of 2 x 1100 complex points), the W_1100
// table and the per-tooth constants stay in LDS for the block's lifetime,
// and each thread keeps the next group's raw words in registers while the
// current group is transformed (non-temporal loads).
#include "internal.h"

namespace cg {
namespace {

constexpr int MX_M = 1100;        // complex points
constexpr int MX_N = 2 * MX_M;    // samples per frame
constexpr int MX_FPB = 2;         // frames per block and group
constexpr int MX_THREADS = 256;

struct cx {
  float x, y;
};

__device__ __forceinline__ cx cmul(cx a, cx b) {
  return {fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x)};
}
__device__ __forceinline__ cx cadd(cx a, cx b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cx csub(cx a, cx b) { return {a.x - b.x, a.y - b.y}; }

// Words per frame in 32-bit units and the complex points one word carries.
template <typename T>
struct Loader;
template <>
struct Loader<int8_t> {
  static constexpr int WORDS = MX_N / 4;  // 550
  __device__ static void put(cx* z, int w, int32_t raw) {
    z[2 * w] = {(float)(int8_t)(raw & 0xff), (float)(int8_t)((raw >> 8) & 0xff)};
    z[2 * w + 1] = {(float)(int8_t)((raw >> 16) & 0xff), (float)(raw >> 24)};
  }
};
template <>
struct Loader<int16_t> {
  static constexpr int WORDS = MX_N / 2;  // 1100
  __device__ static void put(cx* z, int w, int32_t raw) {
    z[w] = {(float)(int16_t)(raw & 0xffff), (float)(raw >> 16)};
  }
};

// One Stockham pass of radix R over the block's frames, src -> dst.
template <int R, int S>
__device__ __forceinline__ void stockham_pass(const cx* __restrict__ src, cx* __restrict__ dst,
                                              const cx* __restrict__ tw) {
  constexpr int NB = MX_M / R;        // butterflies per frame
  constexpr int TWS = MX_M / (S * R);  // twiddle index step
  constexpr int CR = MX_M / R;        // W_R^q = tw[q * CR]
  for (int t = threadIdx.x; t < MX_FPB * NB; t += MX_THREADS) {
    const int f = t / NB;
    const int j = t - f * NB;
    const cx* a = src + f * MX_M;
    cx v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = a[j + r * NB];
    const int kk = j % S;
    if constexpr (S > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) v[r] = cmul(v[r], tw[(kk * r * TWS) % MX_M]);
    }
    cx out[R];
    if constexpr (R == 4) {
      const cx s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
      const cx s13 = cadd(v[1], v[3]), d13 = csub(v[1], v[3]);
      out[0] = cadd(s02, s13);
      out[2] = csub(s02, s13);
      out[1] = {d02.x + d13.y, d02.y - d13.x};  // d02 - i d13
      out[3] = {d02.x - d13.y, d02.y + d13.x};  // d02 + i d13
    } else {
      // odd R: a_r = v_r + v_{R-r}, b_r = v_r - v_{R-r};
      // V_m = v_0 + sum a_r cos(2 pi r m / R) - i sum b_r sin(2 pi r m / R),
      // V_{R-m} = the same with + i
      constexpr int H = (R - 1) / 2;
      cx av[H], bv[H];
      cx v0sum = v[0];
#pragma unroll
      for (int r = 1; r <= H; ++r) {
        av[r - 1] = cadd(v[r], v[R - r]);
        bv[r - 1] = csub(v[r], v[R - r]);
        v0sum = cadd(v0sum, av[r - 1]);
      }
      out[0] = v0sum;
#pragma unroll
      for (int m = 1; m <= H; ++m) {
        cx t1 = v[0], t2 = {0.f, 0.f};
#pragma unroll
        for (int r = 1; r <= H; ++r) {
          const cx w = tw[((r * m) % R) * CR];  // (cos, -sin) of 2 pi r m / R
          t1.x = fmaf(av[r - 1].x, w.x, t1.x);
          t1.y = fmaf(av[r - 1].y, w.x, t1.y);
          t2.x = fmaf(bv[r - 1].x, -w.y, t2.x);
          t2.y = fmaf(bv[r - 1].y, -w.y, t2.y);
        }
        out[m] = {t1.x + t2.y, t1.y - t2.x};      // t1 - i t2
        out[R - m] = {t1.x - t2.y, t1.y + t2.x};  // t1 + i t2
      }
    }
    cx* b = dst + f * MX_M + (j / S) * S * R + kk;
#pragma unroll
    for (int m = 0; m < R; ++m) b[m * S] = out[m];
  }
}

// LDS bytes of the kernel for k teeth: two buffers, the W_1100 table, and per
// tooth the bin, W_2200^bin and 0.5 / reference.
constexpr size_t mx_lds_bytes(int k) {
  return (2 * (size_t)MX_FPB * MX_M + MX_M) * sizeof(cx) + (size_t)k * (sizeof(int) + sizeof(cx) +
                                                                        sizeof(float));
}

template <typename T>
__global__ __launch_bounds__(MX_THREADS) void fft_mixed_kernel(
    const T* __restrict__ frames, int64_t n_frames, const int32_t* __restrict__ bins,
    const float* __restrict__ half_inv_ref, const cx* __restrict__ tw_m,
    const cx* __restrict__ tw_tooth, int k, float* __restrict__ out_mag,
    float* __restrict__ out_y, const int32_t* __restrict__ dev_n) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  cx* buf0 = reinterpret_cast<cx*>(lds);
  cx* buf1 = buf0 + MX_FPB * MX_M;
  cx* tw = buf1 + MX_FPB * MX_M;
  cx* ttw = tw + MX_M;
  int* tbin = reinterpret_cast<int*>(ttw + k);
  float* thr = reinterpret_cast<float*>(tbin + k);
  if (dev_n) {
    const int64_t dn = *dev_n;
    n_frames = dn < n_frames ? dn : n_frames;
  }
  const int64_t ngroups = (n_frames + MX_FPB - 1) / MX_FPB;
  int64_t g = blockIdx.x;
  if (g >= ngroups) return;  // uniform over the block
  for (int e = threadIdx.x; e < MX_M; e += MX_THREADS) tw[e] = tw_m[e];
  for (int i = threadIdx.x; i < k; i += MX_THREADS) {
    ttw[i] = tw_tooth[i];
    tbin[i] = bins[i];
    thr[i] = half_inv_ref[i];
  }
  using L = Loader<T>;
  constexpr int WPT = (MX_FPB * L::WORDS + MX_THREADS - 1) / MX_THREADS;  // words per thread
  const int32_t* words = reinterpret_cast<const int32_t*>(frames);
  const int64_t last = n_frames - 1;
  int32_t raw[WPT];
  auto fetch = [&](int64_t grp) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < WPT; ++u) {
      const int w = threadIdx.x + u * MX_THREADS;  // word of the group
      const int fl = w / L::WORDS;
      const int wf = w - fl * L::WORDS;
      int64_t fr = grp * MX_FPB + (fl < MX_FPB ? fl : MX_FPB - 1);
      fr = fr < last ? fr : last;  // frames past the end read the last one
      raw[u] = w < MX_FPB * L::WORDS
                   ? __builtin_nontemporal_load(words + fr * L::WORDS + wf)
                   : 0;
    }
  };
  fetch(g);
  for (; g < ngroups; g += gridDim.x) {
    __syncthreads();  // previous group's epilogue is done with buf0
#pragma unroll
    for (int u = 0; u < WPT; ++u) {
      const int w = threadIdx.x + u * MX_THREADS;
      if (w < MX_FPB * L::WORDS) {
        const int fl = w / L::WORDS;
        L::put(buf0 + fl * MX_M, w - fl * L::WORDS, raw[u]);
      }
    }
    if (g + gridDim.x < ngroups) fetch(g + gridDim.x);  // next group in flight
    __syncthreads();
    stockham_pass<4, 1>(buf0, buf1, tw);
    __syncthreads();
    stockham_pass<5, 4>(buf1, buf0, tw);
    __syncthreads();
    stockham_pass<5, 20>(buf0, buf1, tw);
    __syncthreads();
    stockham_pass<11, 100>(buf1, buf0, tw);
    __syncthreads();
    // epilogue: the teeth of the group's frames
    for (int t = threadIdx.x; t < MX_FPB * k; t += MX_THREADS) {
      const int fl = t / k;
      const int i = t - fl * k;
      const int64_t frame = g * MX_FPB + fl;
      if (frame >= n_frames) continue;
      const cx* zf = buf0 + fl * MX_M;
      const int b = tbin[i];
      const cx za = zf[b % MX_M];
      const cx zb = zf[(MX_M - b) % MX_M];  // conj taken below
      const cx s = {za.x + zb.x, za.y - zb.y};  // Z[b] + conj Z[M-b]
      const cx d = {za.x - zb.x, za.y + zb.y};  // Z[b] - conj Z[M-b]
      const cx wd = cmul(ttw[i], d);
      const float re = s.x + wd.y, im = s.y - wd.x;  // s - i W d
      const float two_mag = sqrtf(fmaf(re, re, im * im));
      const int64_t o = frame * k + i;
      if (out_mag) out_mag[o] = 0.5f * two_mag;
      if (out_y) out_y[o] = two_mag * thr[i];
    }
  }
}

template <typename T>
int mx_grid_limit(const cg_plan* p) {
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fft_mixed_kernel<T>, MX_THREADS,
                                                   mx_lds_bytes(p->k)) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) !=
          hipSuccess ||
      per_cu <= 0 || cus <= 0)
    return 0;
  return per_cu * cus;
}

template <typename T>
hipError_t launch_mx(const cg_plan* p, const void* frames, int64_t nf, float* out_mag,
                     float* out_y, hipStream_t s, const int32_t* dev_n) {
  int64_t blocks = (nf + MX_FPB - 1) / MX_FPB;
  if (p->fft_blocks > 0 && blocks > p->fft_blocks) blocks = p->fft_blocks;
  if (p->fft_cap > 0 && blocks > p->fft_cap) blocks = p->fft_cap;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  if (blocks == 0) return hipSuccess;
  fft_mixed_kernel<T><<<dim3((unsigned)blocks), dim3(MX_THREADS), mx_lds_bytes(p->k), s>>>(
      static_cast<const T*>(frames), nf, p->d_bins, p->d_half_inv_ref,
      reinterpret_cast<const cx*>(p->d_tw_mixed), reinterpret_cast<const cx*>(p->d_tooth_w),
      p->k, out_mag, out_y, dev_n);
  return hipGetLastError();
}

}  // namespace

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
