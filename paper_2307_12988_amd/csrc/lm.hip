// Batched Levenberg-Marquardt fit of the Lorentzian cavity dip.
//
// Paper, Data Capture and Processing: each normalised spectrum is fitted by a
// Levenberg-Marquardt routine with at most 20 iterations and tolerance 1e-6;
// the fitted centre of the cavity resonance tracks the proof-mass
// displacement (Experimental Setup).  The model is the 4-parameter Lorentzian
// dip f(x) = b (1 - d / (1 + u^2)), u = 2 (x - c) / w, over tooth index x.
//
// gfx950 layout
// -------------
// A wavefront works on 64/G spectra at a time, one per group of G lanes (G = 8
// up to 224 teeth, else 16); lane gl of a group owns teeth i = gl + G q.  Per
// tooth the lane keeps, in registers, the residual r = y - f and the dip term
// g = b d / D (D = 1 + u^2) at the group's current parameters.  A trial point
// is evaluated from the parameter differences, so that every quantity the
// decisions use is computed to FP32 accuracy relative to its own size:
//   du  = u_cur - u_trial             (per-spectrum coefficients from FP64)
//   dD  = D_cur - D_trial = du (2 u_trial + du)
//   dg  = g_trial - g_cur = (d(bd) + dD g_cur) / D_trial
//   df  = f_trial - f_cur = db - dg,  r_trial = r - df,
//   chi2_cur - chi2_trial = sum df (r + r_trial).
// The FP32 residuals are those of the FP32 spectrum plus a rounding of the
// start point's model (a few ulps of b): each step moves them by exactly the
// computed model change, so "chi2 did not increase" and "chi2 fell by at most
// 1e-6 of itself" are decided on a consistent chi2 to within rounding of the
// decrease itself.  Deciding them on two separately rounded FP32 sums instead
// (each off by ~1e-7 of chi2) adds iterations: a decrease of 1e-6 chi2 is
// lost in that noise.  The four Jacobian columns and the 14 normal-equation
// products are FP32 as well; FP64 is used only for the per-spectrum
// parameters and coefficients and the damped 4x4 solve (Cholesky).  DPP
// butterflies inside the group give every lane of the group bit-identical
// sums.  Evaluating a trial point also produces the normal equations there,
// so an accepted step needs no second pass.
//
// A block of up to eight wavefronts (fewer for small launches, so that
// every compute unit gets a block) owns a contiguous range of spectra (one
// chunk per wavefront).  The LM loop body is the same for every iteration, so groups run
// independent fits in lock step: when a group finishes it writes its result
// and takes the next spectrum of the block's range (a wavefront reserves as
// many as it has finished groups with one LDS atomic add), evaluates the new
// start point in the next trip and carries on.  Sharing the range across the
// block's wavefronts evens out their work: a wavefront whose spectra converge
// quickly takes more of them.  The start point is evaluated
// as a trial from the same centre and width with zero depth (where r = y - b
// and g = 0 hold exactly), so one loop body serves both.  A wave exits when
// the block's range is exhausted and all its groups are idle; every fit is
// bounded by max_iter.
//
// Schedule (the paper fixes only the cap and the tolerance): lam0 = 1e-3,
// /10 on accept, *10 on reject; accept when finite, width > 0 and chi2 does
// not increase; converged when an accepted step lowers chi2 by at most
// 1e-6 * chi2_old or chi2 <= 1e-30 (or at the FP32 resolution floor below);
// a non-positive-definite damped matrix stops the fit as singular.
#include <atomic>

#include "fp64.h"
#include "internal.h"
#include "wave.h"

namespace cg {
namespace {

struct Sums {
  float a[10];   // J^T J upper triangle: 00 01 02 03 11 12 13 22 23 33
  float g[4];    // J^T r
  float chi2;    // sum r^2 at the point
  float drop;    // chi2 at the group's current point minus chi2 here
};

// Per-spectrum coefficients of one trial, formed in FP64 and rounded once:
// u at the lane's first tooth and its step per slot at the trial point, the
// same for u_cur - u_trial, and the trial's changes of b d and b.
struct Trial {
  float u0, ustep, du0, dustep, dbd, db, d, b, two_iw;
};

// Sums over the group's teeth at a trial point (a group of G lanes, Q =
// ceil(k / G) slots per lane), and the trial's residuals and dip terms.  The
// arithmetic is the same for every lane; teeth past the last one, which only
// the last slot can hold, contribute exact zeros, and a group whose point is
// not used (idle, or a rejected trial point) simply computes values nobody
// reads, so the loop body has no divergent branches.
//
// The Jacobian columns share per-spectrum factors, which are applied once to
// the reduced sums instead of to every tooth: with u = 2 (x - c) / w,
// D = 1 + u^2, e = 1 / D,
//   df/dc = (-4 b d / w) u e^2,   df/dw = (-2 b d / w) u^2 e^2,
//   df/dd = (-b) e,               df/db = 1 - d e.
// Per tooth only p = u e^2, p u and e enter: the products of the b column
// follow from sums of p, p u, e and r (sum (1 - d e) v = sum v - d sum e v),
// so 13 sums carry the normal equations.
template <int G, int Q>
__device__ __forceinline__ void evaluate(const float (&r)[Q], const float (&g)[Q],
                                         float (&rn)[Q], float (&gn)[Q], int k,
                                         const Trial& t, Sums& s) {
  const int gl = lane_id() & (G - 1);
  // 0 pp, 1 pw, 2 pe, 3 ww, 4 we, 5 ee, 6 p, 7 w, 8 e, 9 pr, 10 wr, 11 er,
  // 12 r, 13 r^2, 14 drop   (w here: p u)
  float acc[15];
#pragma unroll
  for (int j = 0; j < 15; ++j) acc[j] = 0.0f;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    // Two slots at a time between empty asm statements, which keep the
    // compiler from hoisting every slot's first steps (and their registers)
    // to the top of the loop.
    float u = fmaf((float)q, t.ustep, t.u0);
    float du = fmaf((float)q, t.dustep, t.du0);
    if (q % 2 == 0) asm volatile("" : "+v"(u), "+v"(du));
    const float den = fmaf(u, u, 1.0f);
    float e = __builtin_amdgcn_rcpf(den);
    const float dden = du * fmaf(2.0f, u, du);       // D_cur - D_trial
    const float dg = fmaf(dden, g[q], t.dbd) * e;    // g_trial - g_cur
    float df = t.db - dg;                            // f_trial - f_cur
    float rt = r[q] - df;
    gn[q] = g[q] + dg;
    float pc = e * e * u;
    float pw = pc * u;
    if (q == Q - 1) {                                // only the last slot can be partial
      const bool in = gl + G * q < k;
      df = in ? df : 0.0f;
      rt = in ? rt : 0.0f;
      pc = in ? pc : 0.0f;
      pw = in ? pw : 0.0f;
      e = in ? e : 0.0f;
    }
    rn[q] = rt;
    acc[0] = fmaf(pc, pc, acc[0]);
    acc[1] = fmaf(pc, pw, acc[1]);
    acc[2] = fmaf(pc, e, acc[2]);
    acc[3] = fmaf(pw, pw, acc[3]);
    acc[4] = fmaf(pw, e, acc[4]);
    acc[5] = fmaf(e, e, acc[5]);
    acc[6] += pc;
    acc[7] += pw;
    acc[8] += e;
    acc[9] = fmaf(pc, rt, acc[9]);
    acc[10] = fmaf(pw, rt, acc[10]);
    acc[11] = fmaf(e, rt, acc[11]);
    acc[12] += rt;
    acc[13] = fmaf(rt, rt, acc[13]);
    acc[14] = fmaf(df, r[q] + rt, acc[14]);
    if (q % 2 == 1 || q == Q - 1)
      asm volatile(""
                   : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3]), "+v"(acc[4]),
                     "+v"(acc[5]), "+v"(acc[6]), "+v"(acc[7]), "+v"(acc[8]), "+v"(acc[9]),
                     "+v"(acc[10]), "+v"(acc[11]), "+v"(acc[12]), "+v"(acc[13]),
                     "+v"(acc[14]));
  }
  float sm[15];
#pragma unroll
  for (int j = 0; j < 15; ++j) sm[j] = sum_group<G>(acc[j]);
  // column factors: c, w carry al, be (depth included), d carries ga; the b
  // column is 1 - d e
  const float al = -2.0f * t.b * t.two_iw * t.d, be = -t.b * t.two_iw * t.d, ga = -t.b;
  s.a[0] = sm[0] * (al * al);
  s.a[1] = sm[1] * (al * be);
  s.a[2] = sm[2] * (al * ga);
  s.a[3] = al * fmaf(-t.d, sm[2], sm[6]);
  s.a[4] = sm[3] * (be * be);
  s.a[5] = sm[4] * (be * ga);
  s.a[6] = be * fmaf(-t.d, sm[4], sm[7]);
  s.a[7] = sm[5] * (ga * ga);
  s.a[8] = ga * fmaf(-t.d, sm[5], sm[8]);
  s.a[9] = fmaf(-t.d, fmaf(2.0f, sm[8], -t.d * sm[5]), (float)k);
  s.g[0] = sm[9] * al;
  s.g[1] = sm[10] * be;
  s.g[2] = sm[11] * ga;
  s.g[3] = fmaf(-t.d, sm[11], sm[12]);
  s.chi2 = sm[13];
  s.drop = sm[14];
}

// Solve (A + lam diag A) delta = g by Cholesky in FP64; false if the damped
// matrix is not positive definite or the step is not finite.  Straight-line
// code: a failed pivot turns into NaNs that the final test rejects.
__device__ __forceinline__ bool damped_solve(const Sums& s, double lam, double (&delta)[4]) {
  const double sc = 1.0 + lam;
  const double a00 = (double)s.a[0] * sc, a01 = s.a[1], a02 = s.a[2], a03 = s.a[3];
  const double a11 = (double)s.a[4] * sc, a12 = s.a[5], a13 = s.a[6];
  const double a22 = (double)s.a[7] * sc, a23 = s.a[8];
  const double a33 = (double)s.a[9] * sc;
  const double i00 = rsq_d(a00);
  const double l10 = a01 * i00, l20 = a02 * i00, l30 = a03 * i00;
  const double t11 = a11 - l10 * l10;
  const double i11 = rsq_d(t11);
  const double l21 = (a12 - l20 * l10) * i11, l31 = (a13 - l30 * l10) * i11;
  const double t22 = a22 - l20 * l20 - l21 * l21;
  const double i22 = rsq_d(t22);
  const double l32 = (a23 - l30 * l20 - l31 * l21) * i22;
  const double t33 = a33 - l30 * l30 - l31 * l31 - l32 * l32;
  const double i33 = rsq_d(t33);
  const double z0 = (double)s.g[0] * i00;
  const double z1 = ((double)s.g[1] - l10 * z0) * i11;
  const double z2 = ((double)s.g[2] - l20 * z0 - l21 * z1) * i22;
  const double z3 = ((double)s.g[3] - l30 * z0 - l31 * z1 - l32 * z2) * i33;
  delta[3] = z3 * i33;
  delta[2] = (z2 - l32 * delta[3]) * i22;
  delta[1] = (z1 - l21 * delta[2] - l31 * delta[3]) * i11;
  delta[0] = (z0 - l10 * delta[1] - l20 * delta[2] - l30 * delta[3]) * i00;
  const bool pd = a00 > 0.0 && t11 > 0.0 && t22 > 0.0 && t33 > 0.0;
  return pd && isfinite(delta[0]) && isfinite(delta[1]) && isfinite(delta[2]) &&
         isfinite(delta[3]);
}

// A new spectrum: r = y - b and g = 0, the residual and dip term of the
// start point's centre, width and baseline with zero depth (zeros past the
// last tooth).
template <int G, int Q>
__device__ __forceinline__ void load_spectrum(const float* __restrict__ y, int64_t s, int k,
                                              float b, float (&r)[Q], float (&g)[Q]) {
  const int gl = lane_id() & (G - 1);
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int i = gl + G * q;
    r[q] = (q < Q - 1 || i < k) ? y[s * k + i] - b : 0.0f;  // only the last slot can be partial
    g[q] = 0.0f;
  }
}

// The residuals keep the rounding of the model changes they have been moved
// by: a few FP32 ulps of the start point's baseline b0, mostly from the first
// steps.  A fit whose chi2 falls below k (2^-19 b0)^2 (an RMS residual of 16
// ulps of b0) has reached the resolution of this arithmetic and is reported
// converged, as a chi2 <= 1e-30 is in FP64.  Only spectra that the model
// reproduces exactly (noiseless or all-zero) get there: measured spectra sit
// orders of magnitude above it.
__device__ __forceinline__ float resolution_floor(int k, double b0) {
  const float s = 0x1p-19f * (float)fabs(b0);
  return (float)k * s * s;
}

constexpr int LM_WAVES = 8;  // most wavefronts per block

template <int G, int Q>
__global__ __launch_bounds__(64 * LM_WAVES) __attribute__((amdgpu_waves_per_eu(2, 8))) void lm_kernel(
    const float* __restrict__ y, const float* __restrict__ p0, const int32_t* __restrict__ idx,
    const int32_t* __restrict__ count, int64_t nf, int k, int max_iter, int chunk,
    float* __restrict__ params, int32_t* __restrict__ iters, int32_t* __restrict__ status,
    float* __restrict__ chi2_out, int status_code, int32_t* __restrict__ zero_count) {
  constexpr int NG = 64 / G;  // spectra in flight per wave
  // a counter the next kernel on the stream accumulates into (the fallback
  // list after a polish), cleared here so that no kernel has to do only that
  if (zero_count && blockIdx.x == 0 && threadIdx.x == 0) *zero_count = 0;
  __shared__ int s_next;  // next unclaimed spectrum of the block's range (offset)
  const int lane = lane_id();
  const int grp = lane / G;
  const int gl = lane & (G - 1);
  const int wv = threadIdx.x >> 6;
  const int nw = (int)(blockDim.x >> 6);  // wavefronts in this block (1 .. LM_WAVES)
  const int64_t base = (int64_t)blockIdx.x * nw * chunk;
  int64_t n = nf;
  if (count) {
    const int64_t c = *count;
    n = c < nf ? (c < 0 ? 0 : c) : nf;
  }
  if (base >= n) return;  // uniform over the block
  const int64_t span = (int64_t)nw * chunk;
  const int64_t end = base + span < n ? base + span : n;
  if (threadIdx.x == 0) s_next = nw * NG;
  __syncthreads();  // the only block barrier

  int64_t s = base + wv * NG + grp;  // spectrum of this group (>= end: idle)
  bool active = s < end;
  bool fresh = true;
  float r[Q], g[Q], rn[Q], gn[Q];
  // current point (d = 0 until the start point is taken), the start depth,
  // and u = a x + e at the current point
  double c = 0, w = 1, d = 0, b = 0, d_start = 0, lam = 1e-3, ua = 2, ue = 0;
  float floor2 = 0.0f;  // resolution floor of chi2 (see the convergence test)
  int it = 0;
  int64_t fi = 0;  // frame of the current spectrum
  Sums cur;
  if (active) {
    fi = idx ? (int64_t)idx[s] : s;
    c = p0[fi * 4 + 0];
    w = p0[fi * 4 + 1];
    d_start = p0[fi * 4 + 2];
    b = p0[fi * 4 + 3];
    load_spectrum<G, Q>(y, fi, k, (float)b, r, g);
    floor2 = resolution_floor(k, b);
  } else {
#pragma unroll
    for (int q = 0; q < Q; ++q) r[q] = g[q] = 0.0f;
  }
  ua = 2.0 * rcp_d(w);
  ue = -c * ua;

  while (__ballot(active) != 0ull) {
    // 1. damped step for groups past their start point (every group runs the
    //    solve; only those past their start point use it)
    const bool stepping = active && !fresh;
    double delta[4];
    const bool solved = damped_solve(cur, lam, delta) && stepping;
    const double tc = stepping ? c + delta[0] : c, tw = stepping ? w + delta[1] : w;
    const double td = stepping ? d + delta[2] : d_start, tb = stepping ? b + delta[3] : b;
    const bool point_ok = fresh || (solved && isfinite(tc) && isfinite(tw) && isfinite(td) &&
                                    isfinite(tb) && tw > 0.0);
    // 2. evaluation (start point for fresh groups, trial point otherwise);
    //    u = ta x + te at the trial point
    const double ta = 2.0 * rcp_d(tw), te = -tc * ta;
    Trial t;
    t.u0 = (float)fma((double)gl, ta, te);
    t.ustep = (float)(G * ta);
    t.du0 = (float)fma((double)gl, ua - ta, ue - te);
    t.dustep = (float)(G * (ua - ta));
    t.dbd = (float)(tb * td - b * d);
    t.db = (float)(tb - b);
    t.d = (float)td;
    t.b = (float)tb;
    t.two_iw = (float)ta;
    Sums trial;
    evaluate<G, Q>(r, g, rn, gn, k, t, trial);
    // 3. decisions, as selects: the groups of a wave are in different
    //    states, and branches here would only execute every path with copies
    const bool start = active && fresh;
    const bool finite = isfinite(trial.chi2) && isfinite(trial.drop);
    const bool accept = stepping && solved && point_ok && finite && trial.drop >= 0.0f;
    const bool take = start || accept;
    const float old = cur.chi2;
    it = start ? 0 : (stepping ? it + 1 : it);
    lam = start ? 1e-3 : (accept ? lam * 0.1 : ((stepping && solved) ? lam * 10.0 : lam));
    c = take ? tc : c;
    w = take ? tw : w;
    d = take ? td : d;
    b = take ? tb : b;
    ua = take ? ta : ua;
    ue = take ? te : ue;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      r[q] = take ? rn[q] : r[q];
      g[q] = take ? gn[q] : g[q];
    }
#pragma unroll
    for (int j = 0; j < 10; ++j) cur.a[j] = take ? trial.a[j] : cur.a[j];
#pragma unroll
    for (int j = 0; j < 4; ++j) cur.g[j] = take ? trial.g[j] : cur.g[j];
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
    // 4. finished groups report and take the next spectrum of the chunk
    if (done && gl == 0) {
      if (params) {
        params[fi * 4 + 0] = (float)c;
        params[fi * 4 + 1] = (float)w;
        params[fi * 4 + 2] = (float)d;
        params[fi * 4 + 3] = (float)b;
      }
      if (iters) iters[fi] = it;
      if (status) status[fi] = status_code >= 0 ? status_code : st;
      if (chi2_out) chi2_out[fi] = cur.chi2;
    }
    const uint64_t fin = __ballot(done && gl == 0);
    if (fin != 0ull) {
      // reserve one spectrum per finished group from the block's range
      int off = 0;
      if (lane == 0) off = atomicAdd(&s_next, (int)__popcll(fin));
      off = __shfl(off, 0);
      if (done) {
        const uint64_t below = fin & ((1ull << (grp * G)) - 1ull);
        s = base + off + __popcll(below);
        active = s < end;
        fresh = true;
        if (active) {
          fi = idx ? (int64_t)idx[s] : s;
          c = p0[fi * 4 + 0];
          w = p0[fi * 4 + 1];
          d = 0.0;
          d_start = p0[fi * 4 + 2];
          b = p0[fi * 4 + 3];
          load_spectrum<G, Q>(y, fi, k, (float)b, r, g);
          floor2 = resolution_floor(k, b);
          ua = 2.0 * rcp_d(w);
          ue = -c * ua;
        }
      }
    }
  }
}


// The fallback list, one block per 1024 frames: a block flags its frames,
// counts them with a block-wide scan and reserves its place in the list with
// one atomic add on the count, which the polish fit (the kernel before this
// one on the stream) has cleared.  The list order is not specified.
constexpr int FB_THREADS = 256, FB_PER = 4;
__global__ __launch_bounds__(FB_THREADS) void fallback_select_kernel(
    const float* __restrict__ chi2, int64_t nf, float thr2, int32_t* __restrict__ flags,
    int32_t* __restrict__ idx, int32_t* __restrict__ count, const int32_t* __restrict__ dev_n) {
  __shared__ int32_t s_wave[FB_THREADS / 64];
  __shared__ int32_t s_base;
  if (dev_n) {
    const int64_t dn = *dev_n;
    nf = dn < nf ? dn : nf;
  }
  const int64_t f0 = (int64_t)blockIdx.x * FB_THREADS * FB_PER;
  if (f0 >= nf) return;  // uniform over the block
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  uint32_t mask = 0;
#pragma unroll
  for (int i = 0; i < FB_PER; ++i) {
    const int64_t f = f0 + t + (int64_t)FB_THREADS * i;
    if (f < nf) {
      // RMS residual sqrt(chi2 / (k - 4)) > 2 sigma  <=>  chi2 > 4 sigma^2 (k - 4)
      const float c = chi2[f];
      const bool bad = !isfinite(c) || c > thr2;
      flags[f] = bad ? 1 : 0;
      mask |= (uint32_t)bad << i;
    }
  }
  const int cnt = __popc(mask);
  int incl = cnt;  // inclusive scan over the wave
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int v = __shfl_up(incl, d);
    incl += lane >= d ? v : 0;
  }
  if (lane == 63) s_wave[wv] = incl;
  __syncthreads();
  if (t == 0) {
    int total = 0;
#pragma unroll
    for (int w = 0; w < FB_THREADS / 64; ++w) total += s_wave[w];
    s_base = total > 0 ? atomicAdd(count, total) : 0;
  }
  __syncthreads();
  int off = s_base + incl - cnt;
#pragma unroll
  for (int w = 0; w < FB_THREADS / 64; ++w) off += w < wv ? s_wave[w] : 0;
  while (mask) {
    const int i = __builtin_ffs(mask) - 1;
    mask &= mask - 1;
    idx[off++] = (int32_t)(f0 + t + (int64_t)FB_THREADS * i);
  }
}

}  // namespace

hipError_t launch_fallback_select(const float* chi2, int64_t nf, int k, float noise_floor,
                                  int32_t* flags, int32_t* idx, int32_t* count, hipStream_t s,
                                  const int32_t* dev_n) {
  if (nf > 0x7fffffff) return hipErrorInvalidValue;
  const double dof = k > 4 ? (double)(k - 4) : 1.0;
  const float thr2 = (float)(4.0 * (double)noise_floor * (double)noise_floor * dof);
  const int64_t blocks = (nf + FB_THREADS * FB_PER - 1) / (FB_THREADS * FB_PER);
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(fallback_select_kernel, dim3((unsigned)blocks), dim3(FB_THREADS), 0, s, chi2,
                     nf, thr2, flags, idx, count, dev_n);
  return hipGetLastError();
}

// Lanes per spectrum: groups of 8 (eight spectra per wave) while the slots
// per lane stay within 28 (K <= 224), else groups of 16.  Wider waves amortise
// the solve and the decisions over more spectra and shorten the reductions.
int lm_group(int k) { return k <= 224 ? 8 : 16; }

int lm_chunk(int64_t nf, int k, int lanes) {
  // spectra per wave: about four per group, so a group that finishes early
  // has work to take, while keeping at least 2048 waves (two per SIMD) when
  // the batch allows it
  const int ng = 64 / (lanes > 0 ? lanes : lm_group(k));
  int64_t c = nf / 2048;
  if (c > 4 * ng) c = 4 * ng;
  c = (c / ng) * ng;
  if (c < ng) c = ng;
  return (int)c;
}

namespace {

// Compute units of the device plans were last created on (set at plan
// creation, read at launch: launches may be captured into graphs, where no
// device query is made).
std::atomic<int> g_compute_units{0};

template <int G, int Q>
hipError_t launch_lm_gq(const float* y, const float* p0, const int32_t* idx,
                        const int32_t* count, int64_t nf, int k, int max_iter, int chunk,
                        float* params, int32_t* iters, int32_t* status, float* chi2,
                        int32_t status_code, int32_t* zero_count, hipStream_t s) {
  const int nw = fit_waves_per_block((nf + chunk - 1) / chunk);
  const int64_t span = (int64_t)nw * chunk;  // spectra per block
  const int64_t blocks = (nf + span - 1) / span;
  if (blocks > 0x7fffffff || span > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((lm_kernel<G, Q>), dim3((unsigned)blocks), dim3(64 * nw), 0, s, y, p0, idx,
                     count, nf, k, max_iter, chunk, params, iters, status, chi2, status_code,
                     zero_count);
  return hipGetLastError();
}

// The fit kernel is instantiated for every slot count Q = ceil(k / G) <= 28,
// so only its last slot needs masking.
template <int G>
hipError_t launch_lm_g(const float* y, const float* p0, const int32_t* idx,
                       const int32_t* count, int64_t nf, int k, int max_iter, int chunk,
                       float* params, int32_t* iters, int32_t* status, float* chi2,
                       int32_t status_code, int32_t* zero_count, hipStream_t s) {
#define CG_LM_CASE(QV)                                                                   \
  case QV:                                                                               \
    return launch_lm_gq<G, QV>(y, p0, idx, count, nf, k, max_iter, chunk, params, iters, \
                               status, chi2, status_code, zero_count, s);
  switch ((k + G - 1) / G) {
    CG_LM_CASE(1) CG_LM_CASE(2) CG_LM_CASE(3) CG_LM_CASE(4) CG_LM_CASE(5) CG_LM_CASE(6)
    CG_LM_CASE(7) CG_LM_CASE(8) CG_LM_CASE(9) CG_LM_CASE(10) CG_LM_CASE(11) CG_LM_CASE(12)
    CG_LM_CASE(13) CG_LM_CASE(14) CG_LM_CASE(15) CG_LM_CASE(16) CG_LM_CASE(17)
    CG_LM_CASE(18) CG_LM_CASE(19) CG_LM_CASE(20) CG_LM_CASE(21) CG_LM_CASE(22)
    CG_LM_CASE(23) CG_LM_CASE(24) CG_LM_CASE(25) CG_LM_CASE(26) CG_LM_CASE(27)
    CG_LM_CASE(28)
    default:
      return hipErrorInvalidValue;
  }
#undef CG_LM_CASE
}

hipError_t launch_lm_any(const float* y, const float* p0, const int32_t* idx,
                         const int32_t* count, int64_t nf, int k, int max_iter, int chunk,
                         float* params, int32_t* iters, int32_t* status, float* chi2,
                         int32_t status_code, int32_t* zero_count, hipStream_t s, int lanes) {
  if (nf <= 0) return hipSuccess;
  if (lanes != 0 && lanes != 8 && lanes != 16) return hipErrorInvalidValue;
  if (lanes == 0) lanes = lm_group(k);
  if (lanes == 8 && k > 8 * 28) return hipErrorInvalidValue;
  if (lanes == 8)
    return launch_lm_g<8>(y, p0, idx, count, nf, k, max_iter, chunk, params, iters, status,
                          chi2, status_code, zero_count, s);
  return launch_lm_g<16>(y, p0, idx, count, nf, k, max_iter, chunk, params, iters, status,
                         chi2, status_code, zero_count, s);
}

}  // namespace

void set_compute_units(int cus) { g_compute_units.store(cus, std::memory_order_relaxed); }

// Wavefronts per block for a launch of `waves` wavefronts: the block's
// wavefronts share its range of spectra, so blocks are as large as allowed
// while every compute unit still gets a block; small launches use smaller
// blocks spread over more compute units.
int fit_waves_per_block(int64_t waves) {
  const int c = g_compute_units.load(std::memory_order_relaxed);
  const int cus = c > 0 ? c : 256;
  int nw = 8;
  while (nw > 1 && waves < (int64_t)nw * cus) nw >>= 1;
  return nw;
}


hipError_t launch_lm(const float* y, const float* p0, int64_t nf, int k, int max_iter,
                     float* params, int32_t* iters, int32_t* status, float* chi2, hipStream_t s,
                     int chunk, const int32_t* dev_n, int32_t* zero_count, int lanes) {
  if (chunk <= 0) chunk = lm_chunk(nf, k, lanes);
  return launch_lm_any(y, p0, nullptr, dev_n, nf, k, max_iter, chunk, params, iters, status,
                       chi2, -1, zero_count, s, lanes);
}

hipError_t launch_lm_indexed(const float* y, const float* p0, const int32_t* idx,
                             const int32_t* count, int64_t n_cap, int k, int max_iter,
                             float* params, int32_t* iters, int32_t* status, float* chi2,
                             int32_t status_code, hipStream_t s) {
  // The count is only known on the device: one spectrum per group keeps waves
  // busy.  The listed spectra are few and the hardest (they fit for many
  // iterations), so a wave's time is one long dependency chain: 16 lanes per
  // spectrum halve each evaluation's chain against 8, at twice the solve work
  // per spectrum.
  if (n_cap <= 0) return hipSuccess;
  return launch_lm_any(y, p0, idx, count, n_cap, k, max_iter, 4, params, iters, status, chi2,
                       status_code, nullptr, s, 16);
}

}  // namespace cg
