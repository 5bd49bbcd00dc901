// Displacement power spectral density of the fitted centres (Welch) and the
// fit of the mechanical resonance (f, Q).
//
// Paper, Experimental Results and the figure of the power spectral density:
// the centres form a displacement series whose PSD, averaged over seconds to
// minutes, shows the accelerometer's thermomechanical resonance; fitting it
// gives the resonance frequency and the quality factor.
//
// Welch: segments of L samples (L = 2^14 .. 2^17) overlapping by L/2, the
// segment mean removed, periodic Hann window, one-sided density, averaged;
// only a band of bins k_lo .. k_lo + n_bins - 1 is produced.  Each segment's
// real FFT goes through the 1/2-length complex FFT of even/odd-packed samples
// (M = L/2 points) split four-step as M = N1 x 128:
//   Y[k2][n1] = W_M^(n1 k2) sum_n2 z[n1 + N1 n2] W_128^(n2 k2)   (psd_cols)
//   Z[k2 + 128 k1] = sum_n1 Y[k2][n1] W_N1^(n1 k1)               (psd_rows)
// and 2 X[k] = (Z[k] + conj Z[M-k]) - i W_L^k (Z[k] - conj Z[M-k]) at the
// band bins; a block of psd_rows takes the row pair (r, 128 - r), which
// holds both Z[k] and Z[M - k] of its bins.  The column and row FFTs are
// Stockham radix-4 (and one radix-2) passes in LDS.  Segment means come from
// FP64 sums of half-segments (each sample read once).  Segments run in
// chunks; each chunk's per-segment powers are added into FP64 sums in a fixed
// order (groups of 64 consecutive segments, then the groups), and the last
// step scales them into the density.
//
// Resonance fit: one block, FP64 throughout: S(f) = A / ((f0^2 - f^2)^2 +
// (f0 f / Q)^2) + B fitted on ln S over the band by Levenberg-Marquardt
// (lam0 = 1e-3, /10 on accept, *10 on reject, Cholesky, converged when an
// accepted step lowers chi2 by at most tol chi2), parameters (ln A, f0, Q,
// ln B), start point from the peak, its half-width and the median of the
// band's lowest quarter (a bitonic sort of the band in LDS).
#include <cmath>

#include "internal.h"

namespace cg {
namespace {

struct cxf {
  float x, y;
};
__device__ __forceinline__ cxf cmulf(cxf a, cxf b) {
  return {fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x)};
}

constexpr int PSD_N2 = 128;   // column FFT length
constexpr int PSD_COLS = 16;  // columns per block of psd_cols
constexpr int PSD_PAD = 4;    // LDS padding per column

// Stockham passes over `nseq` sequences of P points (sequence s at
// buf + s * stride), ping-ponging between a and b; radix 4 while possible,
// one radix-2 pass if log2 P is odd.  tw holds W_P^e, e < P.  Returns the
// buffer with the result.  Every thread of the block takes part.
template <int P>
__device__ cxf* stockham_pow2(cxf* a, cxf* b, int nseq, int stride, const cxf* tw) {
  int S = 1;
  while (S < P) {
    const int R = (P / S) % 4 == 0 ? 4 : 2;
    const int NB = P / R;
    const int step = P / (S * R);
    for (int t = threadIdx.x; t < nseq * NB; t += blockDim.x) {
      const int sq = t / NB;
      const int j = t - sq * NB;
      const cxf* src = a + sq * stride;
      cxf* dst = b + sq * stride;
      const int kk = j % S;
      if (R == 4) {
        cxf v0 = src[j], v1 = src[j + NB], v2 = src[j + 2 * NB], v3 = src[j + 3 * NB];
        if (S > 1) {
          v1 = cmulf(v1, tw[kk * step]);
          v2 = cmulf(v2, tw[2 * kk * step]);
          v3 = cmulf(v3, tw[3 * kk * step]);
        }
        const cxf s02 = {v0.x + v2.x, v0.y + v2.y}, d02 = {v0.x - v2.x, v0.y - v2.y};
        const cxf s13 = {v1.x + v3.x, v1.y + v3.y}, d13 = {v1.x - v3.x, v1.y - v3.y};
        cxf* o = dst + (j / S) * S * 4 + kk;
        o[0] = {s02.x + s13.x, s02.y + s13.y};
        o[S] = {d02.x + d13.y, d02.y - d13.x};
        o[2 * S] = {s02.x - s13.x, s02.y - s13.y};
        o[3 * S] = {d02.x - d13.y, d02.y + d13.x};
      } else {
        cxf v0 = src[j], v1 = src[j + NB];
        if (S > 1) v1 = cmulf(v1, tw[kk * step]);
        cxf* o = dst + (j / S) * S * 2 + kk;
        o[0] = {v0.x + v1.x, v0.y + v1.y};
        o[S] = {v0.x - v1.x, v0.y - v1.y};
      }
    }
    __syncthreads();
    cxf* t = a;
    a = b;
    b = t;
    S *= R;
  }
  return a;
}

// Per call: Hann window w[t] (periodic), the W_M table and W_L^k for the band.
__global__ void psd_tables_kernel(int L, int k_lo, int n_bins, float* __restrict__ win,
                                  cxf* __restrict__ wm, cxf* __restrict__ wband) {
  const int M = L / 2;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < L; t += gridDim.x * blockDim.x) {
    win[t] = (float)(0.5 - 0.5 * cospi(2.0 * (double)t / (double)L));
    if (t < M) {
      double s, c;
      sincospi(2.0 * (double)t / (double)M, &s, &c);
      wm[t] = {(float)c, (float)-s};
    }
    if (t < n_bins) {
      double s, c;
      sincospi(2.0 * (double)(k_lo + t) / (double)L, &s, &c);
      wband[t] = {(float)c, (float)-s};
    }
  }
}

// FP64 sums of the half-segments (hop = L / 2 samples) h = h0 .. h0 + nh - 1,
// one block each; segment s covers half-segments s and s + 1, so its mean is
// (hsum[s] + hsum[s + 1]) / L and every sample is read once.
__global__ __launch_bounds__(256) void psd_halfsum_kernel(const float* __restrict__ x, int hop,
                                                          int64_t h0, double* __restrict__ hsum) {
  __shared__ double part[4];
  const float2* src = reinterpret_cast<const float2*>(x + (h0 + blockIdx.x) * (int64_t)hop);
  double acc = 0.0;
  for (int t = threadIdx.x; t < hop / 2; t += 256) {
    const float2 v = src[t];
    acc += (double)v.x + (double)v.y;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) hsum[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}

// Column step: block (segment s of the chunk, columns c0 .. c0 + 15).
template <int N1>
__global__ __launch_bounds__(256) void psd_cols_kernel(const float* __restrict__ x, int64_t seg0,
                                                       const double* __restrict__ hsum,
                                                       const float* __restrict__ win,
                                                       const cxf* __restrict__ wm,
                                                       cxf* __restrict__ yg) {
  constexpr int M = N1 * PSD_N2, L = 2 * M, STR = PSD_N2 + PSD_PAD;
  __shared__ cxf bufa[PSD_COLS * STR];
  __shared__ cxf bufb[PSD_COLS * STR];
  __shared__ cxf tw[PSD_N2];
  const int s = blockIdx.y;
  const int c0 = blockIdx.x * PSD_COLS;
  const int64_t start = (seg0 + s) * (int64_t)(L / 2);
  const float m = (float)((hsum[s] + hsum[s + 1]) / (double)L);
  for (int e = threadIdx.x; e < PSD_N2; e += 256) tw[e] = wm[e * N1];  // W_128^e = W_M^(e N1)
  for (int p = threadIdx.x; p < PSD_COLS * PSD_N2; p += 256) {
    const int cl = p % PSD_COLS, n2 = p / PSD_COLS;
    const int n = c0 + cl + N1 * n2;
    const float2 v = *reinterpret_cast<const float2*>(x + start + 2 * n);
    const float2 w = *reinterpret_cast<const float2*>(win + 2 * n);
    bufa[cl * STR + n2] = {(v.x - m) * w.x, (v.y - m) * w.y};
  }
  __syncthreads();
  const cxf* res = stockham_pow2<PSD_N2>(bufa, bufb, PSD_COLS, STR, tw);
  // twiddle W_M^(n1 k2) and store transposed: yg[s][k2][n1]
  for (int p = threadIdx.x; p < PSD_COLS * PSD_N2; p += 256) {
    const int cl = p % PSD_COLS, k2 = p / PSD_COLS;
    const int n1 = c0 + cl;
    const cxf v = cmulf(res[cl * STR + k2], wm[(n1 * k2) % M]);
    yg[(int64_t)s * M + (int64_t)k2 * N1 + n1] = v;
  }
}

// Row step: block (segment s of the chunk, row pair r, 128 - r); band powers
// of the bins whose k mod 128 is r or 128 - r.
template <int N1>
__global__ __launch_bounds__(128) void psd_rows_kernel(const cxf* __restrict__ yg,
                                                       const cxf* __restrict__ wm,
                                                       const cxf* __restrict__ wband, int k_lo,
                                                       int n_bins, float* __restrict__ pseg) {
  constexpr int M = N1 * PSD_N2;
  __shared__ cxf bufa[2 * N1];
  __shared__ cxf bufb[2 * N1];
  __shared__ cxf tw[N1];
  const int s = blockIdx.y;
  const int r = blockIdx.x;  // 0 .. 64
  const int ra = r, rb = (PSD_N2 - r) % PSD_N2;
  for (int e = threadIdx.x; e < N1; e += blockDim.x) tw[e] = wm[e * PSD_N2];  // W_N1^e
  for (int e = threadIdx.x; e < 2 * N1; e += blockDim.x) {
    const int row = e < N1 ? ra : rb;
    bufa[e] = yg[(int64_t)s * M + (int64_t)row * N1 + (e % N1)];
  }
  __syncthreads();
  const cxf* res = stockham_pow2<N1>(bufa, bufb, 2, N1, tw);
  // bins k with k mod 128 in {ra, rb}: the first bin of the band at or above
  // k_lo with residue ra, then every 128th (and the same for rb if distinct)
  const int k_hi = k_lo + n_bins;
  for (int which = 0; which < (ra == rb ? 1 : 2); ++which) {
    const int res_k = which == 0 ? ra : rb;
    const int first = k_lo + ((res_k - k_lo % PSD_N2) + PSD_N2) % PSD_N2;
    for (int k = first + PSD_N2 * (int)threadIdx.x; k < k_hi; k += PSD_N2 * (int)blockDim.x) {
      const int kk = k % M, pp = (M - k % M) % M;
      const int k2 = kk % PSD_N2, k1 = kk / PSD_N2;
      const int p2 = pp % PSD_N2, p1 = pp / PSD_N2;
      const cxf za = res[(k2 == ra ? 0 : N1) + k1];
      const cxf zb = res[(p2 == ra ? 0 : N1) + p1];
      const cxf sm = {za.x + zb.x, za.y - zb.y};
      const cxf df = {za.x - zb.x, za.y + zb.y};
      const cxf wd = cmulf(wband[k - k_lo], df);
      const float re = sm.x + wd.y, im = sm.y - wd.x;  // 2 X[k]
      pseg[(int64_t)s * n_bins + (k - k_lo)] = 0.25f * fmaf(re, re, im * im);
    }
  }
}

// The chunk's per-segment powers into the FP64 sums in a fixed order: groups
// of PSD_GROUP consecutive segments summed in segment order (psd_part), then
// the groups in order (psd_accumulate).
constexpr int PSD_GROUP = 64;
__global__ void psd_part_kernel(const float* __restrict__ pseg, int n_seg, int n_bins,
                                double* __restrict__ part) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_bins) return;
  const int s0 = blockIdx.y * PSD_GROUP;
  const int s1 = s0 + PSD_GROUP < n_seg ? s0 + PSD_GROUP : n_seg;
  double a = 0.0;
  for (int s = s0; s < s1; ++s) a += (double)pseg[(int64_t)s * n_bins + b];
  part[(int64_t)blockIdx.y * n_bins + b] = a;
}

__global__ void psd_accumulate_kernel(const double* __restrict__ part, int n_groups, int n_bins,
                                      double* __restrict__ acc) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_bins) return;
  double a = acc[b];
  for (int g = 0; g < n_groups; ++g) a += part[(int64_t)g * n_bins + b];
  acc[b] = a;
}

__global__ void psd_zero_kernel(double* __restrict__ acc, int n) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < n) acc[b] = 0.0;
}

// density = 2 / (fs sum w^2) * mean power (1 instead of 2 at DC and Nyquist);
// sum w^2 of the periodic Hann window is 3 L / 8 exactly.
__global__ void psd_scale_kernel(const double* __restrict__ acc, int n_bins, int k_lo, int L,
                                 int64_t n_seg, double fs, double* __restrict__ out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_bins) return;
  const int k = k_lo + b;
  const double edge = (k == 0 || k == L / 2) ? 0.5 : 1.0;
  out[b] = acc[b] / (double)n_seg * (2.0 / (fs * (3.0 * (double)L / 8.0))) * edge;
}

// ---------------------------------------------------------------------------
// Resonance fit (one block of 256 threads, FP64).

constexpr int OSC_T = 256;
constexpr int OSC_MAXB = 2048;

// Sums over the block of NV values per thread: butterflies inside each
// wavefront, then the four wavefronts' partial sums through LDS (two
// barriers per call whatever NV is).  Every thread gets every sum.
template <int NV>
__device__ void block_sums(double (&v)[NV], double* red) {
#pragma unroll
  for (int u = 0; u < NV; ++u) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[u] += __shfl_xor(v[u], o);
  }
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int u = 0; u < NV; ++u) red[wv * NV + u] = v[u];
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < NV; ++u)
    v[u] = red[u] + red[NV + u] + red[2 * NV + u] + red[3 * NV + u];
  __syncthreads();
}

// ln S and its gradient with respect to (ln A, f0, Q, ln B) at frequency f
// (ea = A, eb = B).
__device__ __forceinline__ void osc_eval(double f, const double (&p)[4], double ea, double eb,
                                         double& lns, double (&g)[4]) {
  const double f0 = p[1], q = p[2];
  const double dd = f0 * f0 - f * f;
  const double den = dd * dd + (f0 * f / q) * (f0 * f / q);
  const double res = ea / den;
  const double s = res + eb;
  lns = log(s);
  const double dden_df0 = 4.0 * f0 * dd + 2.0 * f0 * f * f / (q * q);
  const double dden_dq = -2.0 * f0 * f0 * f * f / (q * q * q);
  g[0] = res / s;
  g[1] = -res * dden_df0 / den / s;
  g[2] = -res * dden_dq / den / s;
  g[3] = eb / s;
}

// Sums of J^T J (10), J^T r (4) and chi2 over the band at p.
__device__ void osc_sums(const double* __restrict__ lny, double f_first, double df, int nb,
                         const double (&p)[4], double* red, double (&a)[10], double (&g)[4],
                         double& chi2) {
  double v[15] = {0};  // 0..9 J^T J, 10..13 J^T r, 14 chi2
  const double ea = exp(p[0]), eb = exp(p[3]);
  for (int b = threadIdx.x; b < nb; b += OSC_T) {
    double lns, j[4];
    osc_eval(f_first + df * (double)b, p, ea, eb, lns, j);
    const double r = lny[b] - lns;
    v[14] += r * r;
    int o = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      v[10 + u] += j[u] * r;
#pragma unroll
      for (int w = u; w < 4; ++w) v[o++] += j[u] * j[w];
    }
  }
  block_sums<15>(v, red);
#pragma unroll
  for (int o = 0; o < 10; ++o) a[o] = v[o];
#pragma unroll
  for (int u = 0; u < 4; ++u) g[u] = v[10 + u];
  chi2 = v[14];
}

__device__ bool chol4_solve(const double (&a)[10], double lam, const double (&g)[4],
                            double (&d)[4]) {
  // a: 00 01 02 03 11 12 13 22 23 33
  double m[4][4];
  int o = 0;
  for (int u = 0; u < 4; ++u)
    for (int v = u; v < 4; ++v) {
      m[u][v] = a[o];
      m[v][u] = a[o];
      ++o;
    }
  for (int u = 0; u < 4; ++u) m[u][u] *= 1.0 + lam;
  double l[4][4] = {{0}};
  for (int i = 0; i < 4; ++i) {
    for (int jj = 0; jj <= i; ++jj) {
      double sum = m[i][jj];
      for (int kk = 0; kk < jj; ++kk) sum -= l[i][kk] * l[jj][kk];
      if (i == jj) {
        if (!(sum > 0.0)) return false;
        l[i][i] = sqrt(sum);
      } else {
        l[i][jj] = sum / l[jj][jj];
      }
    }
  }
  double z[4];
  for (int i = 0; i < 4; ++i) {
    double sum = g[i];
    for (int kk = 0; kk < i; ++kk) sum -= l[i][kk] * z[kk];
    z[i] = sum / l[i][i];
  }
  for (int i = 3; i >= 0; --i) {
    double sum = z[i];
    for (int kk = i + 1; kk < 4; ++kk) sum -= l[kk][i] * d[kk];
    d[i] = sum / l[i][i];
  }
  for (int i = 0; i < 4; ++i)
    if (!isfinite(d[i])) return false;
  return true;
}

__global__ __launch_bounds__(OSC_T) void osc_fit_kernel(const double* __restrict__ psd, int nb,
                                                        double f_first, double df, int max_iter,
                                                        double tol, double* __restrict__ out) {
  __shared__ double lny[OSC_MAXB];
  __shared__ double srt[OSC_MAXB];
  __shared__ double val[OSC_MAXB];
  __shared__ double red[4 * 15];
  __shared__ double sp[4];
  __shared__ int pk[4];
  int npow = 1;
  while (npow < nb) npow <<= 1;
  for (int b = threadIdx.x; b < npow; b += OSC_T) {
    if (b < nb) {
      const double v = psd[b];
      lny[b] = log(v);
      srt[b] = v;
      val[b] = v;
    } else {
      srt[b] = INFINITY;
    }
  }
  __syncthreads();
  // bitonic sort of the band (ascending) for the floor estimate
  for (int size = 2; size <= npow; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < npow; i += OSC_T) {
        const int jx = i ^ stride;
        if (jx > i) {
          const bool up = (i & size) == 0;
          const double u = srt[i], v = srt[jx];
          if ((u > v) == up) {
            srt[i] = v;
            srt[jx] = u;
          }
        }
      }
      __syncthreads();
    }
  }
  // the peak: the first bin holding the band's largest value
  {
    int ib = threadIdx.x < nb ? (int)threadIdx.x : 0;
    for (int b = threadIdx.x + OSC_T; b < nb; b += OSC_T)
      if (val[b] > val[ib]) ib = b;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const int oth = __shfl_xor(ib, o);
      if (val[oth] > val[ib] || (val[oth] == val[ib] && oth < ib)) ib = oth;
    }
    if ((threadIdx.x & 63) == 0) pk[threadIdx.x >> 6] = ib;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    // start point: peak, floor, half-width
    int ipk = pk[0];
    for (int w = 1; w < 4; ++w)
      if (val[pk[w]] > val[ipk] || (val[pk[w]] == val[ipk] && pk[w] < ipk)) ipk = pk[w];
    const int qn = nb / 4 > 1 ? nb / 4 : 1;
    const double floor_b = (qn % 2 == 1) ? srt[qn / 2] : 0.5 * (srt[qn / 2 - 1] + srt[qn / 2]);
    const double half = floor_b + 0.5 * (val[ipk] - floor_b);
    int lo = ipk, hi = ipk;
    while (lo > 0 && val[lo] > half) --lo;
    while (hi < nb - 1 && val[hi] > half) ++hi;
    const double f0 = f_first + df * (double)ipk;
    double width = df * (double)(hi - lo);
    width = width > df ? width : df;
    double q = f0 / width;
    q = q > 1.0 ? q : 1.0;
    double ex = val[ipk] - floor_b;
    ex = ex > 1e-300 ? ex : 1e-300;
    const double a = ex * f0 * f0 * f0 * f0 / (q * q);
    sp[0] = log(a);
    sp[1] = f0;
    sp[2] = q;
    sp[3] = log(floor_b > 1e-300 ? floor_b : 1e-300);
  }
  __syncthreads();
  double p[4] = {sp[0], sp[1], sp[2], sp[3]};
  double a[10], g[4], chi2;
  osc_sums(lny, f_first, df, nb, p, red, a, g, chi2);
  double lam = 1e-3;
  int it = 0, status = CG_FIT_MAX_ITER;
  while (it < max_iter) {
    ++it;
    double d[4];
    const bool ok_solve = chol4_solve(a, lam, g, d);  // same in every thread
    if (!ok_solve) {
      status = CG_FIT_SINGULAR;
      break;
    }
    double t[4] = {p[0] + d[0], p[1] + d[1], p[2] + d[2], p[3] + d[3]};
    const bool ok_pt = isfinite(t[0]) && isfinite(t[1]) && isfinite(t[2]) && isfinite(t[3]) &&
                       t[1] > 0.0 && t[2] > 0.0;
    double at[10], gt[4], ct = INFINITY;
    if (ok_pt) osc_sums(lny, f_first, df, nb, t, red, at, gt, ct);
    if (!(ok_pt && isfinite(ct) && ct <= chi2)) {
      lam *= 10.0;
      continue;
    }
    const double drop = chi2 - ct, old = chi2;
    for (int u = 0; u < 4; ++u) {
      p[u] = t[u];
      g[u] = gt[u];
    }
    for (int o = 0; o < 10; ++o) a[o] = at[o];
    chi2 = ct;
    lam /= 10.0;
    if (drop <= tol * old) {
      status = CG_FIT_CONVERGED;
      break;
    }
  }
  if (threadIdx.x == 0) {
    out[0] = p[0];
    out[1] = p[1];
    out[2] = p[2];
    out[3] = p[3];
    out[4] = chi2;
    out[5] = (double)it;
    out[6] = (double)status;
  }
}

template <int N1>
hipError_t run_chunk(const float* x, int64_t seg0, int nseg, int k_lo, int n_bins,
                     const float* win, const cxf* wm, const cxf* wband, double* hsum, cxf* yg,
                     float* pseg, double* part, double* acc, hipStream_t s) {
  constexpr int L = 2 * N1 * PSD_N2;
  const int groups = (nseg + PSD_GROUP - 1) / PSD_GROUP;
  hipLaunchKernelGGL(psd_halfsum_kernel, dim3(nseg + 1), dim3(256), 0, s, x, L / 2, seg0, hsum);
  hipLaunchKernelGGL((psd_cols_kernel<N1>), dim3(N1 / PSD_COLS, nseg), dim3(256), 0, s, x, seg0,
                     hsum, win, wm, yg);
  hipLaunchKernelGGL((psd_rows_kernel<N1>), dim3(PSD_N2 / 2 + 1, nseg), dim3(128), 0, s, yg, wm,
                     wband, k_lo, n_bins, pseg);
  hipLaunchKernelGGL(psd_part_kernel, dim3((n_bins + 255) / 256, groups), dim3(256), 0, s, pseg,
                     nseg, n_bins, part);
  hipLaunchKernelGGL(psd_accumulate_kernel, dim3((n_bins + 255) / 256), dim3(256), 0, s, part,
                     groups, n_bins, acc);
  return hipGetLastError();
}

size_t a256p(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

size_t psd_workspace_bytes(int64_t chunk_segments, int seg_len, int n_bins) {
  const size_t M = (size_t)seg_len / 2;
  const size_t groups = ((size_t)chunk_segments + PSD_GROUP - 1) / PSD_GROUP;
  return a256p(sizeof(float) * (size_t)seg_len) + a256p(sizeof(cxf) * M) +
         a256p(sizeof(cxf) * (size_t)n_bins) + a256p(sizeof(double) * (size_t)n_bins) +
         a256p(sizeof(double) * ((size_t)chunk_segments + 1)) +
         a256p(sizeof(cxf) * M * (size_t)chunk_segments) +
         a256p(sizeof(float) * (size_t)n_bins * (size_t)chunk_segments) +
         a256p(sizeof(double) * (size_t)n_bins * groups);
}

hipError_t launch_psd(const float* x, int64_t n, double fs, int seg_len, int k_lo, int n_bins,
                      double* out, void* ws, int64_t chunk_segments, hipStream_t s) {
  const int M = seg_len / 2;
  const int64_t hop = seg_len / 2;
  const int64_t n_seg = (n - seg_len) / hop + 1;
  char* c = static_cast<char*>(ws);
  float* win = reinterpret_cast<float*>(c);
  c += a256p(sizeof(float) * (size_t)seg_len);
  cxf* wm = reinterpret_cast<cxf*>(c);
  c += a256p(sizeof(cxf) * (size_t)M);
  cxf* wband = reinterpret_cast<cxf*>(c);
  c += a256p(sizeof(cxf) * (size_t)n_bins);
  double* acc = reinterpret_cast<double*>(c);
  c += a256p(sizeof(double) * (size_t)n_bins);
  double* hsum = reinterpret_cast<double*>(c);
  c += a256p(sizeof(double) * ((size_t)chunk_segments + 1));
  cxf* yg = reinterpret_cast<cxf*>(c);
  c += a256p(sizeof(cxf) * (size_t)M * (size_t)chunk_segments);
  float* pseg = reinterpret_cast<float*>(c);
  c += a256p(sizeof(float) * (size_t)n_bins * (size_t)chunk_segments);
  double* part = reinterpret_cast<double*>(c);
  hipLaunchKernelGGL(psd_tables_kernel, dim3((seg_len + 255) / 256), dim3(256), 0, s, seg_len,
                     k_lo, n_bins, win, wm, wband);
  hipLaunchKernelGGL(psd_zero_kernel, dim3((n_bins + 255) / 256), dim3(256), 0, s, acc, n_bins);
  hipError_t e = hipGetLastError();
  for (int64_t seg0 = 0; seg0 < n_seg && e == hipSuccess; seg0 += chunk_segments) {
    const int nseg = (int)(n_seg - seg0 < chunk_segments ? n_seg - seg0 : chunk_segments);
    switch (seg_len) {
      case 16384:
        e = run_chunk<64>(x, seg0, nseg, k_lo, n_bins, win, wm, wband, hsum, yg, pseg, part, acc, s);
        break;
      case 32768:
        e = run_chunk<128>(x, seg0, nseg, k_lo, n_bins, win, wm, wband, hsum, yg, pseg, part, acc, s);
        break;
      case 65536:
        e = run_chunk<256>(x, seg0, nseg, k_lo, n_bins, win, wm, wband, hsum, yg, pseg, part, acc, s);
        break;
      case 131072:
        e = run_chunk<512>(x, seg0, nseg, k_lo, n_bins, win, wm, wband, hsum, yg, pseg, part, acc, s);
        break;
      default:
        e = hipErrorInvalidValue;
    }
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(psd_scale_kernel, dim3((n_bins + 255) / 256), dim3(256), 0, s, acc, n_bins,
                     k_lo, seg_len, n_seg, fs, out);
  return hipGetLastError();
}

hipError_t launch_osc_fit(const double* psd, int n_bins, double f_first, double df,
                          int max_iter, double tol, double* out, hipStream_t s) {
  if (n_bins < 8 || n_bins > OSC_MAXB) return hipErrorInvalidValue;
  hipLaunchKernelGGL(osc_fit_kernel, dim3(1), dim3(OSC_T), 0, s, psd, n_bins, f_first, df,
                     max_iter, tol, out);
  return hipGetLastError();
}

}  // namespace cg
