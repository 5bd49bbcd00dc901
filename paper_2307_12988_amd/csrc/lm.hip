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
// evaluation each lane computes model, residual and chi2 in FP64 (so the chi2
// comparisons and the 1e-6 relative-decrease test see the same values an
// FP64 reference sees) and the four Jacobian columns and the 14
// normal-equation products in FP32; DPP butterflies inside the group give
// every lane of the group bit-identical sums.  The damped 4x4 system is solved
// per group by a Cholesky factorisation in FP64.  Evaluating a trial point
// also produces the normal equations there, so an accepted step needs no
// second pass.
//
// A wave owns a contiguous chunk of spectra.  The LM loop body is the same for
// every iteration, so groups run independent fits in lock step: when a group
// finishes it writes its result and takes the next spectrum of the chunk (the
// hand-out index is wave-uniform, advanced with a ballot), evaluates the new
// start point in the next trip and carries on.  A wave exits when its chunk is
// exhausted and all its groups are idle; every fit is bounded by max_iter.
//
// Schedule (the paper fixes only the cap and the tolerance): lam0 = 1e-3,
// /10 on accept, *10 on reject; accept when finite, width > 0 and chi2 does
// not increase; converged when an accepted step lowers chi2 by at most
// 1e-6 * chi2_old or chi2 <= 1e-30; a non-positive-definite damped matrix
// stops the fit as singular.
#include "fp64.h"
#include "internal.h"
#include "wave.h"

namespace cg {
namespace {

struct Sums {
  float a[10];   // J^T J upper triangle: 00 01 02 03 11 12 13 22 23 33
  float g[4];    // J^T r
  double chi2;
};

// Sums over the group's teeth at one parameter point (a group of G lanes,
// Q = ceil(k / G) slots per lane).  The arithmetic is the same for every lane; teeth past the last
// one, which only the last slot can hold, contribute exact zeros, and a
// group whose point is not used (idle, or a rejected trial point) simply
// computes values nobody reads, so the loop body has no divergent branches.
//
// The Jacobian columns share per-spectrum factors, which are applied once to
// the reduced sums instead of to every tooth: with u = 2 (x - c) / w,
// D = 1 + u^2, s = d / D^2,
//   df/dc = (-4 b / w) s u,   df/dw = (-2 b / w) s u^2,
//   df/dd = (-b) / D,         df/db = 1 - d / D.
//
// Per tooth the FP64 part is u (from the lane's first tooth plus a constant
// offset), D, 1 / D and the residual r = (y - b) + (b d) / D, which is
// y - f(x) rounded differently; the FP32 Jacobian factors start from FP32
// copies of the same quantities.
template <int G, int Q>
__device__ __forceinline__ void evaluate(const float (&yv)[Q], int k, double c, double w,
                                         double d, double b, Sums& s) {
  const int gl = lane_id() & (G - 1);
  float acc[14];
#pragma unroll
  for (int j = 0; j < 14; ++j) acc[j] = 0.0f;
  double chi2 = 0.0;
  const double two_iw = 2.0 * rcp_d(w);
  const double u0 = fma((double)gl, two_iw, -c * two_iw);  // u at tooth gl
  const double bd = b * d;
  const float two_iwf = (float)two_iw, u0f = (float)u0, df = (float)d;
  const double step = (double)G * two_iw;
  double u_prev = u0;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    // The empty asm statements pin pairs of slots in program order: the u of
    // the pair's first slot passes through one before the pair's arithmetic
    // and the sums pass through one after the pair.  Each u is the previous
    // one plus the tooth step (one FP64 add; an fma from u0 with the slot's
    // offset needs a register copy of u0 first, as the offset is a literal).  Left alone, the compiler evaluates the FP64 part of
    // every slot first and keeps all of it live (about 100 extra VGPRs); two
    // slots at a time give the scheduler two independent chains.
    const int i = gl + G * q;
    double u;
    if (q % 2 == 0) {
      u = q == 0 ? u0 : u_prev + step;
      asm volatile("" : "+v"(u));
    } else {
      u = u_prev + step;
    }
    u_prev = u;
    const double den = fma(u, u, 1.0);
    const double inv = rcp1_d(den);
    double r = fma(bd, inv, (double)yv[q] - b);
    const float invf = (float)inv;
    const float uf = fmaf((float)(G * q), two_iwf, u0f);
    const float qf = df * invf;  // d / D
    float jc = qf * invf * uf;   // s u
    float jw = jc * uf;          // s u^2
    float jd = invf;             // 1 / D
    float jb = 1.0f - qf;        // 1 - d / D
    if (q == Q - 1) {            // only the last slot can be partial
      const bool in = i < k;
      r = in ? r : 0.0;
      jc = in ? jc : 0.0f;
      jw = in ? jw : 0.0f;
      jd = in ? jd : 0.0f;
      jb = in ? jb : 0.0f;
    }
    const float rf = (float)r;
    chi2 = fma(r, r, chi2);
    acc[0] = fmaf(jc, jc, acc[0]);
    acc[1] = fmaf(jc, jw, acc[1]);
    acc[2] = fmaf(jc, jd, acc[2]);
    acc[3] = fmaf(jc, jb, acc[3]);
    acc[4] = fmaf(jw, jw, acc[4]);
    acc[5] = fmaf(jw, jd, acc[5]);
    acc[6] = fmaf(jw, jb, acc[6]);
    acc[7] = fmaf(jd, jd, acc[7]);
    acc[8] = fmaf(jd, jb, acc[8]);
    acc[9] = fmaf(jb, jb, acc[9]);
    acc[10] = fmaf(jc, rf, acc[10]);
    acc[11] = fmaf(jw, rf, acc[11]);
    acc[12] = fmaf(jd, rf, acc[12]);
    acc[13] = fmaf(jb, rf, acc[13]);
    if (q % 2 == 1 || q == Q - 1)
      asm volatile(""
                 : "+v"(chi2), "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3]),
                   "+v"(acc[4]), "+v"(acc[5]), "+v"(acc[6]), "+v"(acc[7]), "+v"(acc[8]),
                   "+v"(acc[9]), "+v"(acc[10]), "+v"(acc[11]), "+v"(acc[12]), "+v"(acc[13]));
  }
  float sum[14];
#pragma unroll
  for (int j = 0; j < 14; ++j) sum[j] = sum_group<G>(acc[j]);
  // column factors: c, w, d carry al, be, ga; b carries 1
  const float bf = (float)b;
  const float al = -2.0f * bf * two_iwf, be = -bf * two_iwf, ga = -bf;
  s.a[0] = sum[0] * (al * al);
  s.a[1] = sum[1] * (al * be);
  s.a[2] = sum[2] * (al * ga);
  s.a[3] = sum[3] * al;
  s.a[4] = sum[4] * (be * be);
  s.a[5] = sum[5] * (be * ga);
  s.a[6] = sum[6] * be;
  s.a[7] = sum[7] * (ga * ga);
  s.a[8] = sum[8] * ga;
  s.a[9] = sum[9];
  s.g[0] = sum[10] * al;
  s.g[1] = sum[11] * be;
  s.g[2] = sum[12] * ga;
  s.g[3] = sum[13];
  s.chi2 = sum_group<G>(chi2);
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

template <int G, int Q>
__device__ __forceinline__ void load_spectrum(const float* __restrict__ y, int64_t s, int k,
                                              float (&yv)[Q]) {
  const int gl = lane_id() & (G - 1);
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int i = gl + G * q;
    yv[q] = (q < Q - 1 || i < k) ? y[s * k + i] : 0.0f;  // only the last slot can be partial
  }
}

template <int G, int Q>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8))) void lm_kernel(const float* __restrict__ y,
                                                 const float* __restrict__ p0,
                                                 const int32_t* __restrict__ idx,
                                                 const int32_t* __restrict__ count, int64_t nf,
                                                 int k, int max_iter, int chunk,
                                                 float* __restrict__ params,
                                                 int32_t* __restrict__ iters,
                                                 int32_t* __restrict__ status,
                                                 float* __restrict__ chi2_out, int status_code,
                                                 int32_t* __restrict__ zero_count) {
  constexpr int NG = 64 / G;  // spectra in flight per wave
  // a counter the next kernel on the stream accumulates into (the fallback
  // list after a polish), cleared here so that no kernel has to do only that
  if (zero_count && blockIdx.x == 0 && threadIdx.x == 0) *zero_count = 0;
  const int lane = lane_id();
  const int grp = lane / G;
  const int gl = lane & (G - 1);
  const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t base = wave * chunk;
  int64_t n = nf;
  if (count) {
    const int64_t c = *count;
    n = c < nf ? (c < 0 ? 0 : c) : nf;
  }
  if (base >= n) return;
  const int64_t end = base + chunk < n ? base + chunk : n;

  int64_t s = base + grp;  // spectrum of this group (>= end: idle)
  int64_t next = base + NG;  // wave-uniform hand-out index
  bool active = s < end;
  bool fresh = true;
  float yv[Q];
  double c = 0, w = 1, d = 0, b = 0, lam = 1e-3;
  int it = 0;
  int64_t fi = 0;  // frame of the current spectrum
  Sums cur;
  if (active) {
    fi = idx ? (int64_t)idx[s] : s;
    load_spectrum<G, Q>(y, fi, k, yv);
    c = p0[fi * 4 + 0];
    w = p0[fi * 4 + 1];
    d = p0[fi * 4 + 2];
    b = p0[fi * 4 + 3];
  } else {
#pragma unroll
    for (int q = 0; q < Q; ++q) yv[q] = 0.0f;
  }

  while (__ballot(active) != 0ull) {
    // 1. damped step for groups past their start point (every group runs the
    //    solve; only those past their start point use it)
    const bool stepping = active && !fresh;
    double delta[4];
    const bool solved = damped_solve(cur, lam, delta) && stepping;
    const double tc = stepping ? c + delta[0] : c, tw = stepping ? w + delta[1] : w;
    const double td = stepping ? d + delta[2] : d, tb = stepping ? b + delta[3] : b;
    const bool point_ok = fresh || (solved && isfinite(tc) && isfinite(tw) && isfinite(td) &&
                                    isfinite(tb) && tw > 0.0);
    // 2. evaluation (start point for fresh groups, trial point otherwise)
    Sums trial;
    evaluate<G, Q>(yv, k, tc, tw, td, tb, trial);
    // 3. decisions, as selects: the four groups of a wave are in different
    //    states, and branches here would only execute every path with copies
    const bool start = active && fresh;
    const bool accept = stepping && solved && point_ok && isfinite(trial.chi2) &&
                        trial.chi2 <= cur.chi2;
    const bool take = start || accept;
    const double old = cur.chi2;
    it = start ? 0 : (stepping ? it + 1 : it);
    lam = start ? 1e-3 : (accept ? lam * 0.1 : ((stepping && solved) ? lam * 10.0 : lam));
    c = take ? tc : c;
    w = take ? tw : w;
    d = take ? td : d;
    b = take ? tb : b;
#pragma unroll
    for (int j = 0; j < 10; ++j) cur.a[j] = take ? trial.a[j] : cur.a[j];
#pragma unroll
    for (int j = 0; j < 4; ++j) cur.g[j] = take ? trial.g[j] : cur.g[j];
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
      if (chi2_out) chi2_out[fi] = (float)cur.chi2;
    }
    const uint64_t fin = __ballot(done && gl == 0);
    if (fin != 0ull) {
      if (done) {
        const uint64_t below = fin & ((1ull << (grp * G)) - 1ull);
        s = next + __popcll(below);
        active = s < end;
        fresh = true;
        if (active) {
          fi = idx ? (int64_t)idx[s] : s;
          load_spectrum<G, Q>(y, fi, k, yv);
          c = p0[fi * 4 + 0];
          w = p0[fi * 4 + 1];
          d = p0[fi * 4 + 2];
          b = p0[fi * 4 + 3];
        }
      }
      next += __popcll(fin);
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

template <int G, int Q>
hipError_t launch_lm_gq(const float* y, const float* p0, const int32_t* idx,
                        const int32_t* count, int64_t nf, int k, int max_iter, int chunk,
                        float* params, int32_t* iters, int32_t* status, float* chi2,
                        int32_t status_code, int32_t* zero_count, hipStream_t s) {
  const int64_t waves = (nf + chunk - 1) / chunk;
  const int64_t blocks = (waves + 3) / 4;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((lm_kernel<G, Q>), dim3((unsigned)blocks), dim3(256), 0, s, y, p0, idx,
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
