// Box-constrained Levenberg-Marquardt fit of the asymmetric Fano cavity dip:
// the paper's own fit.
//
// Paper, Data Capture and Processing: every spectrum is fitted with a
// five-parameter asymmetric Fano lineshape, at most 20 iterations and
// tolerance 1e-6; only the centre is free, the scale and the extent are held
// within about +-10 % of pre-computed averages, and the asymmetry and the
// width are fixed to values measured beforehand for the device.
//
//   f(x) = b (1 - d (1 + u / q)^2 / (1 + u^2)),   u = 2 (x - c) / w,
//
// over tooth index x, with c free, d in [dlo, dhi], b in [blo, bhi], w and q
// fixed.  The start point is the 7x7-median centre with d and b at their
// averages.
//
// gfx950 layout: as the Lorentzian fit (lm.hip) -- a group of G lanes per
// spectrum (8 up to 224 teeth, else 16), 64/G spectra per wavefront, a
// block's (up to eight) wavefronts sharing its range of spectra through an LDS
// counter, lane gl owns teeth gl + G q; model, residual and chi2 per tooth in
// FP64 (the fit has one free positional parameter and no width change, so
// the Lorentzian fit's differential FP32 form would save nothing here), the three
// Jacobian columns and the nine normal-equation sums in FP32 with their
// per-spectrum factors applied to the reduced sums, DPP reductions giving
// bit-identical sums in every lane of a group, and the damped 3x3 system
// solved by an FP64 Cholesky factorisation.  The box: a boxed parameter that
// sits on a bound while J^T r points out of the box is held for the step
// (its row and column of the damped matrix become the identity, its
// right-hand side zero), and every trial point is clipped into the box
// before it is evaluated.  Schedule as the Lorentzian fit: lam0 = 1e-3, /10
// on accept, *10 on reject, accept when finite and chi2 does not increase,
// converged when an accepted step lowers chi2 by at most 1e-6 chi2.
#include "fp64.h"
#include "internal.h"
#include "wave.h"

namespace cg {
namespace {

struct FanoSums {
  float a[6];  // J^T J upper triangle over (c, d, b): 00 01 02 11 12 22
  float g[3];  // J^T r
  double chi2;
};

struct FanoArgs {
  double w, two_iw, inv_q;     // fixed width, 2 / w, 1 / q
  double dbar, bbar;           // averages (start values of d and b)
  double dlo, dhi, blo, bhi;   // box
};

// Sums over the group's teeth at (c, d, b).  With D = 1 + u^2, s = 1 + u/q,
// g = s^2 / D and h = (s / q - u g) / D:
//   df/dc = (4 b d / w) h,   df/dd = -b g,   df/db = 1 - d g;
// the column factors 4 b d / w and -b are applied to the reduced sums.
template <int G, int Q>
__device__ __forceinline__ void evaluate_fano(const float (&yv)[Q], int k, double c, double d,
                                              double b, const FanoArgs& fa, FanoSums& s) {
  const int gl = lane_id() & (G - 1);
  float acc[9];
#pragma unroll
  for (int j = 0; j < 9; ++j) acc[j] = 0.0f;
  double chi2 = 0.0;
  const double u0 = fma((double)gl, fa.two_iw, -c * fa.two_iw);  // u at tooth gl
  const double step = (double)G * fa.two_iw;
  const double bd = b * d;
  const float two_iwf = (float)fa.two_iw, u0f = (float)u0, iqf = (float)fa.inv_q;
  const float df = (float)d;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int i = gl + G * q;
    // pairs of slots pinned in program order (see the Lorentzian fit): each
    // pair's FP64 chain starts from a u that passes an empty asm statement
    double u = fma((double)q, step, u0);
    if (q % 2 == 0) asm volatile("" : "+v"(u));
    const double den = fma(u, u, 1.0);
    const double inv = rcp1_d(den);
    const double sq = fma(u, fa.inv_q, 1.0);
    const double gg = sq * sq * inv;
    double r = fma(bd, gg, (double)yv[q] - b);
    const float uf = fmaf((float)(G * q), two_iwf, u0f);
    const float invf = (float)inv;
    const float sf = fmaf(uf, iqf, 1.0f);
    const float gf = (float)gg;
    float jc = invf * fmaf(sf, iqf, -uf * gf);  // h
    float jd = gf;                               // g
    float jb = fmaf(-df, gf, 1.0f);              // 1 - d g
    if (q == Q - 1) {  // only the last slot can be partial
      const bool in = i < k;
      r = in ? r : 0.0;
      jc = in ? jc : 0.0f;
      jd = in ? jd : 0.0f;
      jb = in ? jb : 0.0f;
    }
    const float rf = (float)r;
    chi2 = fma(r, r, chi2);
    acc[0] = fmaf(jc, jc, acc[0]);
    acc[1] = fmaf(jc, jd, acc[1]);
    acc[2] = fmaf(jc, jb, acc[2]);
    acc[3] = fmaf(jd, jd, acc[3]);
    acc[4] = fmaf(jd, jb, acc[4]);
    acc[5] = fmaf(jb, jb, acc[5]);
    acc[6] = fmaf(jc, rf, acc[6]);
    acc[7] = fmaf(jd, rf, acc[7]);
    acc[8] = fmaf(jb, rf, acc[8]);
    if (q % 2 == 1 || q == Q - 1)
      asm volatile(""
                   : "+v"(chi2), "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3]),
                     "+v"(acc[4]), "+v"(acc[5]), "+v"(acc[6]), "+v"(acc[7]), "+v"(acc[8]));
  }
  float sum[9];
#pragma unroll
  for (int j = 0; j < 9; ++j) sum[j] = sum_group<G>(acc[j]);
  const float al = (float)(2.0 * bd * fa.two_iw), be = (float)(-b);
  s.a[0] = sum[0] * (al * al);
  s.a[1] = sum[1] * (al * be);
  s.a[2] = sum[2] * al;
  s.a[3] = sum[3] * (be * be);
  s.a[4] = sum[4] * be;
  s.a[5] = sum[5];
  s.g[0] = sum[6] * al;
  s.g[1] = sum[7] * be;
  s.g[2] = sum[8];
  s.chi2 = sum_group<G>(chi2);
}

// (A + lam diag A) delta = g over (c, d, b) by Cholesky in FP64, with the
// held parameters' rows and columns replaced by the identity and their
// right-hand sides by zero.  Straight-line code; false when the damped
// matrix is not positive definite or the step is not finite.
__device__ __forceinline__ bool fano_solve(const FanoSums& s, double lam, bool hold_d,
                                           bool hold_b, double (&delta)[3]) {
  const double sc = 1.0 + lam;
  const double a00 = (double)s.a[0] * sc;
  const double a01 = hold_d ? 0.0 : (double)s.a[1];
  const double a02 = hold_b ? 0.0 : (double)s.a[2];
  const double a11 = hold_d ? 1.0 : (double)s.a[3] * sc;
  const double a12 = (hold_d || hold_b) ? 0.0 : (double)s.a[4];
  const double a22 = hold_b ? 1.0 : (double)s.a[5] * sc;
  const double g0 = s.g[0];
  const double g1 = hold_d ? 0.0 : (double)s.g[1];
  const double g2 = hold_b ? 0.0 : (double)s.g[2];
  const double i00 = rsq_d(a00);
  const double l10 = a01 * i00, l20 = a02 * i00;
  const double t11 = a11 - l10 * l10;
  const double i11 = rsq_d(t11);
  const double l21 = (a12 - l20 * l10) * i11;
  const double t22 = a22 - l20 * l20 - l21 * l21;
  const double i22 = rsq_d(t22);
  const double z0 = g0 * i00;
  const double z1 = (g1 - l10 * z0) * i11;
  const double z2 = (g2 - l20 * z0 - l21 * z1) * i22;
  delta[2] = z2 * i22;
  delta[1] = (z1 - l21 * delta[2]) * i11;
  delta[0] = (z0 - l10 * delta[1] - l20 * delta[2]) * i00;
  const bool pd = a00 > 0.0 && t11 > 0.0 && t22 > 0.0;
  return pd && isfinite(delta[0]) && isfinite(delta[1]) && isfinite(delta[2]);
}

template <int G, int Q>
__device__ __forceinline__ void load_row(const float* __restrict__ y, int64_t s, int k,
                                         float (&yv)[Q]) {
  const int gl = lane_id() & (G - 1);
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int i = gl + G * q;
    yv[q] = (q < Q - 1 || i < k) ? y[s * k + i] : 0.0f;
  }
}

__device__ __forceinline__ double clampd(double v, double lo, double hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

// A wave fits a contiguous chunk of spectra; groups that finish take the next
// spectrum of the chunk (wave-uniform hand-out index), as in the Lorentzian
// fit.  Start point: p0[f][0] as the centre, d and b at their averages.
constexpr int FANO_WAVES = 8;  // most wavefronts per block (they share the block's range)

template <int G, int Q>
__global__ __launch_bounds__(64 * FANO_WAVES) __attribute__((amdgpu_waves_per_eu(3, 8))) void fano_kernel(
    const float* __restrict__ y, const float* __restrict__ p0, int64_t nf, int k, int max_iter,
    int chunk, FanoArgs fa, float* __restrict__ params, int32_t* __restrict__ iters,
    int32_t* __restrict__ status, float* __restrict__ chi2_out,
    const int32_t* __restrict__ dev_n) {
  constexpr int NG = 64 / G;
  __shared__ int s_next;  // next unclaimed spectrum of the block's range (offset)
  const int lane = lane_id();
  const int grp = lane / G;
  const int gl = lane & (G - 1);
  const int wv = threadIdx.x >> 6;
  const int nw = (int)(blockDim.x >> 6);  // wavefronts in this block
  const int64_t base = (int64_t)blockIdx.x * nw * chunk;
  int64_t n = nf;
  if (dev_n) {
    const int64_t dn = *dev_n;
    n = dn < nf ? (dn < 0 ? 0 : dn) : nf;
  }
  if (base >= n) return;  // uniform over the block
  const int64_t span = (int64_t)nw * chunk;
  const int64_t end = base + span < n ? base + span : n;
  if (threadIdx.x == 0) s_next = nw * NG;
  __syncthreads();  // the only block barrier

  int64_t s = base + wv * NG + grp;
  bool active = s < end;
  bool fresh = true;
  float yv[Q];
  const double d_start = clampd(fa.dbar, fa.dlo, fa.dhi), b_start = clampd(fa.bbar, fa.blo, fa.bhi);
  double c = 0, d = d_start, b = b_start, lam = 1e-3;
  int it = 0;
  FanoSums cur = {};
  if (active) {
    load_row<G, Q>(y, s, k, yv);
    c = p0[s * 4 + 0];
  } else {
#pragma unroll
    for (int q = 0; q < Q; ++q) yv[q] = 0.0f;
  }

  while (__ballot(active) != 0ull) {
    const bool stepping = active && !fresh;
    // hold a boxed parameter on its bound while the gradient points outward
    const bool hold_d = (d <= fa.dlo && cur.g[1] < 0.0f) || (d >= fa.dhi && cur.g[1] > 0.0f);
    const bool hold_b = (b <= fa.blo && cur.g[2] < 0.0f) || (b >= fa.bhi && cur.g[2] > 0.0f);
    double delta[3];
    const bool solved = fano_solve(cur, lam, hold_d, hold_b, delta) && stepping;
    const double tc = stepping ? c + delta[0] : c;
    const double td = stepping ? clampd(d + delta[1], fa.dlo, fa.dhi) : d;
    const double tb = stepping ? clampd(b + delta[2], fa.blo, fa.bhi) : b;
    const bool point_ok = fresh || (solved && isfinite(tc) && isfinite(td) && isfinite(tb));
    FanoSums trial;
    evaluate_fano<G, Q>(yv, k, tc, td, tb, fa, trial);
    const bool start = active && fresh;
    const bool accept = stepping && solved && point_ok && isfinite(trial.chi2) &&
                        trial.chi2 <= cur.chi2;
    const bool take = start || accept;
    const double old = cur.chi2;
    it = start ? 0 : (stepping ? it + 1 : it);
    lam = start ? 1e-3 : (accept ? lam * 0.1 : ((stepping && solved) ? lam * 10.0 : lam));
    c = take ? tc : c;
    d = take ? td : d;
    b = take ? tb : b;
#pragma unroll
    for (int j = 0; j < 6; ++j) cur.a[j] = take ? trial.a[j] : cur.a[j];
#pragma unroll
    for (int j = 0; j < 3; ++j) cur.g[j] = take ? trial.g[j] : cur.g[j];
    cur.chi2 = take ? trial.chi2 : cur.chi2;
    fresh = active ? false : fresh;
    const bool start_bad = start && !isfinite(trial.chi2);
    const bool start_exact = start && !start_bad && trial.chi2 <= 1e-30;
    const bool singular = stepping && !solved;
    const bool conv = accept && (old - trial.chi2 <= 1e-6 * old || trial.chi2 <= 1e-30);
    const bool capped = stepping && !singular && !conv && it >= max_iter;
    const bool done = start_bad || start_exact || singular || conv || capped;
    const int st = (start_bad || singular) ? CG_FIT_SINGULAR
                                           : ((start_exact || conv) ? CG_FIT_CONVERGED
                                                                    : CG_FIT_MAX_ITER);
    if (done && gl == 0) {
      if (params) {
        params[s * 4 + 0] = (float)c;
        params[s * 4 + 1] = (float)fa.w;
        params[s * 4 + 2] = (float)d;
        params[s * 4 + 3] = (float)b;
      }
      if (iters) iters[s] = it;
      if (status) status[s] = st;
      if (chi2_out) chi2_out[s] = (float)cur.chi2;
    }
    const uint64_t fin = __ballot(done && gl == 0);
    if (fin != 0ull) {
      // one spectrum per finished group from the block's range
      int off = 0;
      if (lane == 0) off = atomicAdd(&s_next, (int)__popcll(fin));
      off = __shfl(off, 0);
      if (done) {
        const uint64_t below = fin & ((1ull << (grp * G)) - 1ull);
        s = base + off + __popcll(below);
        active = s < end;
        fresh = true;
        d = d_start;
        b = b_start;
        if (active) {
          load_row<G, Q>(y, s, k, yv);
          c = p0[s * 4 + 0];
        }
      }
    }
  }
}

template <int G, int Q>
hipError_t launch_fano_gq(const float* y, const float* p0, int64_t nf, int k, int max_iter,
                          int chunk, const FanoArgs& fa, float* params, int32_t* iters,
                          int32_t* status, float* chi2, hipStream_t s, const int32_t* dev_n) {
  const int nw = fit_waves_per_block((nf + chunk - 1) / chunk);
  const int64_t span = (int64_t)nw * chunk;  // spectra per block
  const int64_t blocks = (nf + span - 1) / span;
  if (blocks > 0x7fffffff || span > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((fano_kernel<G, Q>), dim3((unsigned)blocks), dim3(64 * nw), 0, s, y, p0, nf, k,
                     max_iter, chunk, fa, params, iters, status, chi2, dev_n);
  return hipGetLastError();
}

template <int G>
hipError_t launch_fano_g(const float* y, const float* p0, int64_t nf, int k, int max_iter,
                         int chunk, const FanoArgs& fa, float* params, int32_t* iters,
                         int32_t* status, float* chi2, hipStream_t s, const int32_t* dev_n) {
#define CG_FANO_CASE(QV) \
  case QV:               \
    return launch_fano_gq<G, QV>(y, p0, nf, k, max_iter, chunk, fa, params, iters, status, chi2, s, dev_n);
  switch ((k + G - 1) / G) {
    CG_FANO_CASE(1) CG_FANO_CASE(2) CG_FANO_CASE(3) CG_FANO_CASE(4) CG_FANO_CASE(5)
    CG_FANO_CASE(6) CG_FANO_CASE(7) CG_FANO_CASE(8) CG_FANO_CASE(9) CG_FANO_CASE(10)
    CG_FANO_CASE(11) CG_FANO_CASE(12) CG_FANO_CASE(13) CG_FANO_CASE(14) CG_FANO_CASE(15)
    CG_FANO_CASE(16) CG_FANO_CASE(17) CG_FANO_CASE(18) CG_FANO_CASE(19) CG_FANO_CASE(20)
    CG_FANO_CASE(21) CG_FANO_CASE(22) CG_FANO_CASE(23) CG_FANO_CASE(24) CG_FANO_CASE(25)
    CG_FANO_CASE(26) CG_FANO_CASE(27) CG_FANO_CASE(28)
    default:
      return hipErrorInvalidValue;
  }
#undef CG_FANO_CASE
}

}  // namespace

hipError_t launch_fano(const cg_plan* p, const float* y, const float* p0, int64_t nf,
                       int max_iter, float* params, int32_t* iters, int32_t* status, float* chi2,
                       hipStream_t s, const int32_t* dev_n) {
  if (nf <= 0) return hipSuccess;
  if (!p->fano_set) return hipErrorInvalidValue;
  FanoArgs fa;
  fa.w = p->fano_w;
  fa.two_iw = 2.0 / p->fano_w;
  fa.inv_q = 1.0 / p->fano_q;
  fa.dbar = p->fano_dbar;
  fa.bbar = p->fano_bbar;
  fa.dlo = 0.9 * p->fano_dbar;
  fa.dhi = 1.1 * p->fano_dbar;
  fa.blo = 0.9 * p->fano_bbar;
  fa.bhi = 1.1 * p->fano_bbar;
  const int lanes = p->lm_lanes > 0 ? p->lm_lanes : lm_group(p->k);
  if (lanes == 8 && p->k > 8 * 28) return hipErrorInvalidValue;
  const int chunk = p->lm_chunk > 0 ? p->lm_chunk : lm_chunk(nf, p->k, lanes);
  if (lanes == 8)
    return launch_fano_g<8>(y, p0, nf, p->k, max_iter, chunk, fa, params, iters, status, chi2, s,
                            dev_n);
  return launch_fano_g<16>(y, p0, nf, p->k, max_iter, chunk, fa, params, iters, status, chi2, s,
                           dev_n);
}

}  // namespace cg
