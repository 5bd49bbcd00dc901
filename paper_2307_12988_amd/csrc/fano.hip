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
// counter, lane gl owns teeth gl + G q.  Per tooth everything is FP32 in the
// Lorentzian fit's differential form: each lane keeps the residual r and
// 1/D of the current point, and a trial point is evaluated from the
// parameter differences, so the chi2 decrease the decisions use is exact to
// FP32 rounding of itself.  With u = 2 (x - c) / w, D = 1 + u^2,
// s = 1 + u/q, g = s^2 / D, and du = u_cur - u_trial (the same for every
// tooth: the width is fixed), D_cur - D_trial = du (2 u + du) and
// s_cur^2 - s_trial^2 = (du/q) (2 s + du/q), so
//   g_trial - g_cur = (s^2 (D_cur - D_trial) - D (s_cur^2 - s^2)) / (D D_cur)
// at the trial's u, s, D, and the model change is
//   f_trial - f_cur = db - (d(bd) g_trial + (bd)_cur (g_trial - g_cur)).
// The three Jacobian columns and the nine normal-equation sums are FP32 with
// their per-spectrum factors applied to the reduced sums, DPP reductions give
// bit-identical sums in every lane of a group, and the damped 3x3 system is
// solved by an FP64 Cholesky factorisation.  The box: a boxed parameter that
// sits on a bound while J^T r points out of the box is held for the step
// (its row and column of the damped matrix become the identity, its
// right-hand side zero), and every trial point is clipped into the box
// before it is evaluated.  Schedule as the Lorentzian fit: lam0 = 1e-3, /10
// on accept, *10 on reject, accept when finite and chi2 does not increase,
// converged when an accepted step lowers chi2 by at most 1e-6 chi2 (or chi2
// is below the FP32 resolution floor, see fano_floor).
#include "fp64.h"
#include "internal.h"
#include "wave.h"

namespace cg {
namespace {

struct FanoSums {
  float a[6];  // J^T J upper triangle over (c, d, b): 00 01 02 11 12 22
  float g[3];  // J^T r
  float chi2;  // sum r^2 at the point
  float drop;  // chi2 at the group's current point minus chi2 here
};

// Per-spectrum coefficients of one trial, formed in FP64 and rounded once.
struct FanoTrial {
  float u0, ustep;      // u at the lane's first tooth and per slot (trial point)
  float du, duq;        // u_cur - u_trial (every tooth) and du / q
  float dbd, db, bd0;   // d(bd), db, (bd) at the current point
  float d, b;           // trial extent and scale
};

struct FanoArgs {
  double w, two_iw, inv_q;     // fixed width, 2 / w, 1 / q
  double dbar, bbar;           // averages (start values of d and b)
  double dlo, dhi, blo, bhi;   // box
};

// Sums over the group's teeth at a trial point, and the trial's residuals
// and 1/D.  Jacobian: with h = (s / q - u g) / D,
//   df/dc = (4 b d / w) h,   df/dd = -b g,   df/db = 1 - d g;
// the column factors 4 b d / w and -b are applied to the reduced sums.
template <int G, int Q>
__device__ __forceinline__ void evaluate_fano(const float (&r)[Q], const float (&ic)[Q],
                                              float (&rn)[Q], float (&inv_n)[Q], int k,
                                              const FanoTrial& t, const FanoArgs& fa,
                                              FanoSums& s) {
  const int gl = lane_id() & (G - 1);
  float acc[11];
#pragma unroll
  for (int j = 0; j < 11; ++j) acc[j] = 0.0f;
  const float iq = (float)fa.inv_q;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    // pairs of slots pinned in program order (see the Lorentzian fit)
    float u = fmaf((float)q, t.ustep, t.u0);
    if (q % 2 == 0) asm volatile("" : "+v"(u));
    const float den = fmaf(u, u, 1.0f);
    float e = __builtin_amdgcn_rcpf(den);                   // 1 / D
    const float sv = fmaf(u, iq, 1.0f);                     // s
    const float s2 = sv * sv;
    const float dden = t.du * fmaf(2.0f, u, t.du);          // D_cur - D_trial
    const float ds2 = t.duq * fmaf(2.0f, sv, t.duq);        // s_cur^2 - s^2
    const float dg = fmaf(s2, dden, -den * ds2) * e * ic[q];  // g_trial - g_cur
    const float g = s2 * e;
    float df = t.db - fmaf(t.dbd, g, t.bd0 * dg);           // f_trial - f_cur
    float rt = r[q] - df;
    inv_n[q] = e;
    float jc = e * fmaf(sv, iq, -u * g);                    // h
    float jd = g;
    float jb = fmaf(-t.d, g, 1.0f);                         // 1 - d g
    if (q == Q - 1) {  // only the last slot can be partial
      const bool in = gl + G * q < k;
      df = in ? df : 0.0f;
      rt = in ? rt : 0.0f;
      jc = in ? jc : 0.0f;
      jd = in ? jd : 0.0f;
      jb = in ? jb : 0.0f;
    }
    rn[q] = rt;
    acc[0] = fmaf(jc, jc, acc[0]);
    acc[1] = fmaf(jc, jd, acc[1]);
    acc[2] = fmaf(jc, jb, acc[2]);
    acc[3] = fmaf(jd, jd, acc[3]);
    acc[4] = fmaf(jd, jb, acc[4]);
    acc[5] = fmaf(jb, jb, acc[5]);
    acc[6] = fmaf(jc, rt, acc[6]);
    acc[7] = fmaf(jd, rt, acc[7]);
    acc[8] = fmaf(jb, rt, acc[8]);
    acc[9] = fmaf(rt, rt, acc[9]);
    acc[10] = fmaf(df, r[q] + rt, acc[10]);
    if (q % 2 == 1 || q == Q - 1)
      asm volatile(""
                   : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3]), "+v"(acc[4]),
                     "+v"(acc[5]), "+v"(acc[6]), "+v"(acc[7]), "+v"(acc[8]), "+v"(acc[9]),
                     "+v"(acc[10]));
  }
  float sum[11];
#pragma unroll
  for (int j = 0; j < 11; ++j) sum[j] = sum_group<G>(acc[j]);
  const float al = 2.0f * t.b * t.d * (float)fa.two_iw, be = -t.b;
  s.a[0] = sum[0] * (al * al);
  s.a[1] = sum[1] * (al * be);
  s.a[2] = sum[2] * al;
  s.a[3] = sum[3] * (be * be);
  s.a[4] = sum[4] * be;
  s.a[5] = sum[5];
  s.g[0] = sum[6] * al;
  s.g[1] = sum[7] * be;
  s.g[2] = sum[8];
  s.chi2 = sum[9];
  s.drop = sum[10];
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

// A new spectrum: r = y - b and 1/D = 0, the residual and the dip term's
// factor of the start centre and scale with zero extent (zeros past the last
// tooth).
template <int G, int Q>
__device__ __forceinline__ void load_row(const float* __restrict__ y, int64_t s, int k, float b,
                                         float (&r)[Q], float (&ic)[Q]) {
  const int gl = lane_id() & (G - 1);
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int i = gl + G * q;
    r[q] = (q < Q - 1 || i < k) ? y[s * k + i] - b : 0.0f;  // only the last slot can be partial
    ic[q] = 0.0f;
  }
}

// The stored residuals carry a few FP32 ulps of the scale b0 from the model
// changes they were moved by; a fit whose chi2 falls below k (2^-19 b0)^2
// (16 ulps RMS) has reached this arithmetic's resolution and is reported
// converged, as the Lorentzian fit does.
__device__ __forceinline__ float fano_floor(int k, double b0) {
  const float s = 0x1p-19f * (float)fabs(b0);
  return (float)k * s * s;
}

__device__ __forceinline__ double clampd(double v, double lo, double hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

// A wave fits a contiguous chunk of spectra; groups that finish take the next
// spectrum of the chunk (wave-uniform hand-out index), as in the Lorentzian
// fit.  Start point: p0[f][0] as the centre, d and b at their averages,
// evaluated as a trial from the same centre and scale with zero extent (whose
// residuals y - b and zero dip term need no evaluation).
constexpr int FANO_WAVES = 8;  // most wavefronts per block (they share the block's range)

template <int G, int Q>
__global__ __launch_bounds__(64 * FANO_WAVES) __attribute__((amdgpu_waves_per_eu(2, 8))) void fano_kernel(
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
  float r[Q], ic[Q], rn[Q], in_n[Q];
  const double d_start = clampd(fa.dbar, fa.dlo, fa.dhi), b_start = clampd(fa.bbar, fa.blo, fa.bhi);
  const float floor2 = fano_floor(k, b_start);  // resolution floor of chi2
  // current point (d = 0 until the start point is taken)
  double c = 0, d = 0, b = b_start, lam = 1e-3;
  int it = 0;
  FanoSums cur = {};
  if (active) {
    load_row<G, Q>(y, s, k, (float)b_start, r, ic);
    c = p0[s * 4 + 0];
  } else {
#pragma unroll
    for (int q = 0; q < Q; ++q) r[q] = ic[q] = 0.0f;
  }

  while (__ballot(active) != 0ull) {
    // 1. damped step for groups past their start point
    const bool stepping = active && !fresh;
    // hold a boxed parameter on its bound while the gradient points outward
    const bool hold_d = (d <= fa.dlo && cur.g[1] < 0.0f) || (d >= fa.dhi && cur.g[1] > 0.0f);
    const bool hold_b = (b <= fa.blo && cur.g[2] < 0.0f) || (b >= fa.bhi && cur.g[2] > 0.0f);
    double delta[3];
    const bool solved = fano_solve(cur, lam, hold_d, hold_b, delta) && stepping;
    const double tc = stepping ? c + delta[0] : c;
    const double td = stepping ? clampd(d + delta[1], fa.dlo, fa.dhi) : d_start;
    const double tb = stepping ? clampd(b + delta[2], fa.blo, fa.bhi) : b;
    const bool point_ok = fresh || (solved && isfinite(tc) && isfinite(td) && isfinite(tb));
    // 2. evaluation (start point for fresh groups, trial point otherwise)
    const double te = -tc * fa.two_iw, du = (tc - c) * fa.two_iw;
    FanoTrial t;
    t.u0 = (float)fma((double)gl, fa.two_iw, te);
    t.ustep = (float)(G * fa.two_iw);
    t.du = (float)du;
    t.duq = (float)(du * fa.inv_q);
    t.dbd = (float)(tb * td - b * d);
    t.db = (float)(tb - b);
    t.bd0 = (float)(b * d);
    t.d = (float)td;
    t.b = (float)tb;
    FanoSums trial;
    evaluate_fano<G, Q>(r, ic, rn, in_n, k, t, fa, trial);
    // 3. decisions, as selects (the groups of a wave are in different states)
    const bool start = active && fresh;
    const bool finite = isfinite(trial.chi2) && isfinite(trial.drop);
    const bool accept = stepping && solved && point_ok && finite && trial.drop >= 0.0f;
    const bool take = start || accept;
    const float old = cur.chi2;
    it = start ? 0 : (stepping ? it + 1 : it);
    lam = start ? 1e-3 : (accept ? lam * 0.1 : ((stepping && solved) ? lam * 10.0 : lam));
    c = take ? tc : c;
    d = take ? td : d;
    b = take ? tb : b;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      r[q] = take ? rn[q] : r[q];
      ic[q] = take ? in_n[q] : ic[q];
    }
#pragma unroll
    for (int j = 0; j < 6; ++j) cur.a[j] = take ? trial.a[j] : cur.a[j];
#pragma unroll
    for (int j = 0; j < 3; ++j) cur.g[j] = take ? trial.g[j] : cur.g[j];
    cur.chi2 = take ? trial.chi2 : cur.chi2;
    fresh = active ? false : fresh;
    const bool start_bad = start && !finite;
    const bool start_exact = start && !start_bad && trial.chi2 <= 1e-30f;
    const bool singular = stepping && !solved;
    const bool conv =
        accept && (trial.drop <= 1e-6f * old || trial.chi2 <= 1e-30f || trial.chi2 <= floor2);
    const bool capped = stepping && !singular && !conv && it >= max_iter;
    const bool done = start_bad || start_exact || singular || conv || capped;
    const int st = (start_bad || singular) ? CG_FIT_SINGULAR
                                           : ((start_exact || conv) ? CG_FIT_CONVERGED
                                                                    : CG_FIT_MAX_ITER);
    // 4. finished groups report and take the next spectrum of the range
    if (done && gl == 0) {
      if (params) {
        params[s * 4 + 0] = (float)c;
        params[s * 4 + 1] = (float)fa.w;
        params[s * 4 + 2] = (float)d;
        params[s * 4 + 3] = (float)b;
      }
      if (iters) iters[s] = it;
      if (status) status[s] = st;
      if (chi2_out) chi2_out[s] = cur.chi2;
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
        d = 0.0;
        b = b_start;
        if (active) {
          load_row<G, Q>(y, s, k, (float)b_start, r, ic);
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
