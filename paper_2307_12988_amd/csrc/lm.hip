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
// A wavefront works on four spectra at a time, one per group of 16 lanes (one
// DPP row); lane gl of a group owns teeth i = gl + 16 q.  Per evaluation each
// lane computes model, residual and chi2 in FP64 (so the chi2 comparisons and
// the 1e-6 relative-decrease test see the same values an FP64 reference sees)
// and the four Jacobian columns and the 14 normal-equation products in FP32;
// 16-lane DPP butterflies give every lane of the group bit-identical sums.  The
// damped 4x4 system is solved per group by a Cholesky factorisation in FP64.
// Evaluating a trial point also produces the normal equations there, so an
// accepted step needs no second pass.
//
// A wave owns a contiguous chunk of spectra.  The LM loop body is the same for
// every iteration, so groups run independent fits in lock step: when a group
// finishes it writes its result and takes the next spectrum of the chunk (the
// hand-out index is wave-uniform, advanced with a ballot), evaluates the new
// start point in the next trip and carries on.  A wave exits when its chunk is
// exhausted and all four groups are idle; every fit is bounded by max_iter.
//
// Schedule (the paper fixes only the cap and the tolerance): lam0 = 1e-3,
// /10 on accept, *10 on reject; accept when finite, width > 0 and chi2 does
// not increase; converged when an accepted step lowers chi2 by at most
// 1e-6 * chi2_old or chi2 <= 1e-30; a non-positive-definite damped matrix
// stops the fit as singular.
#include "internal.h"
#include "wave.h"

namespace cg {
namespace {

struct Sums {
  float a[10];   // J^T J upper triangle: 00 01 02 03 11 12 13 22 23 33
  float g[4];    // J^T r
  double chi2;
};

__device__ __forceinline__ double rcp_d(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

__device__ __forceinline__ double rsq_d(double x) {
  double r = __builtin_amdgcn_rsq(x);
  // Newton for 1/sqrt: r <- r (3 - x r^2) / 2
  double h = 0.5 * x;
  r = r * fma(-h * r, r, 1.5);
  r = r * fma(-h * r, r, 1.5);
  return r;
}

template <int Q>
__device__ __forceinline__ void evaluate(const float (&yv)[Q], int k, bool live, double c,
                                         double w, double d, double b, Sums& s) {
  const int gl = lane_id() & 15;
  float acc[14];
#pragma unroll
  for (int j = 0; j < 14; ++j) acc[j] = 0.0f;
  double chi2 = 0.0;
  const double two_iw = 2.0 * rcp_d(w);
  const float two_iwf = (float)two_iw;
  const float four_iwf = 2.0f * two_iwf;
  const float bf = (float)b;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int i = gl + 16 * q;
    if (live && i < k) {
      const double u = ((double)i - c) * two_iw;
      const double den = fma(u, u, 1.0);
      const double inv = rcp_d(den);
      const double qd = d * inv;
      const double f = fma(-b, qd, b);
      const double r = (double)yv[q] - f;
      chi2 = fma(r, r, chi2);
      const float uf = (float)u, invf = (float)inv, qf = (float)qd, rf = (float)r;
      const float t = bf * qf * invf;          // b d / D^2
      const float jc = -t * uf * four_iwf;     // -4 b d u / (w D^2)
      const float jw = -t * uf * uf * two_iwf; // -2 b d u^2 / (w D^2)
      const float jd = -bf * invf;             // -b / D
      const float jb = 1.0f - qf;              // 1 - d / D
      acc[0] += jc * jc;
      acc[1] += jc * jw;
      acc[2] += jc * jd;
      acc[3] += jc * jb;
      acc[4] += jw * jw;
      acc[5] += jw * jd;
      acc[6] += jw * jb;
      acc[7] += jd * jd;
      acc[8] += jd * jb;
      acc[9] += jb * jb;
      acc[10] += jc * rf;
      acc[11] += jw * rf;
      acc[12] += jd * rf;
      acc[13] += jb * rf;
    }
  }
#pragma unroll
  for (int j = 0; j < 10; ++j) s.a[j] = sum16(acc[j]);
#pragma unroll
  for (int j = 0; j < 4; ++j) s.g[j] = sum16(acc[10 + j]);
  s.chi2 = sum16(chi2);
}

// Solve (A + lam diag A) delta = g by Cholesky in FP64; false if the damped
// matrix is not positive definite.
__device__ __forceinline__ bool damped_solve(const Sums& s, double lam, double (&delta)[4]) {
  const double sc = 1.0 + lam;
  const double a00 = (double)s.a[0] * sc, a01 = s.a[1], a02 = s.a[2], a03 = s.a[3];
  const double a11 = (double)s.a[4] * sc, a12 = s.a[5], a13 = s.a[6];
  const double a22 = (double)s.a[7] * sc, a23 = s.a[8];
  const double a33 = (double)s.a[9] * sc;
  if (!(a00 > 0.0)) return false;
  const double i00 = rsq_d(a00);
  const double l10 = a01 * i00, l20 = a02 * i00, l30 = a03 * i00;
  const double t11 = a11 - l10 * l10;
  if (!(t11 > 0.0)) return false;
  const double i11 = rsq_d(t11);
  const double l21 = (a12 - l20 * l10) * i11, l31 = (a13 - l30 * l10) * i11;
  const double t22 = a22 - l20 * l20 - l21 * l21;
  if (!(t22 > 0.0)) return false;
  const double i22 = rsq_d(t22);
  const double l32 = (a23 - l30 * l20 - l31 * l21) * i22;
  const double t33 = a33 - l30 * l30 - l31 * l31 - l32 * l32;
  if (!(t33 > 0.0)) return false;
  const double i33 = rsq_d(t33);
  const double z0 = (double)s.g[0] * i00;
  const double z1 = ((double)s.g[1] - l10 * z0) * i11;
  const double z2 = ((double)s.g[2] - l20 * z0 - l21 * z1) * i22;
  const double z3 = ((double)s.g[3] - l30 * z0 - l31 * z1 - l32 * z2) * i33;
  delta[3] = z3 * i33;
  delta[2] = (z2 - l32 * delta[3]) * i22;
  delta[1] = (z1 - l21 * delta[2] - l31 * delta[3]) * i11;
  delta[0] = (z0 - l10 * delta[1] - l20 * delta[2] - l30 * delta[3]) * i00;
  return isfinite(delta[0]) && isfinite(delta[1]) && isfinite(delta[2]) && isfinite(delta[3]);
}

template <int Q>
__device__ __forceinline__ void load_spectrum(const float* __restrict__ y, int64_t s, int k,
                                              float (&yv)[Q]) {
  const int gl = lane_id() & 15;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int i = gl + 16 * q;
    yv[q] = i < k ? y[s * k + i] : 0.0f;
  }
}

template <int Q>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8))) void lm_kernel(const float* __restrict__ y,
                                                 const float* __restrict__ p0,
                                                 const int32_t* __restrict__ idx,
                                                 const int32_t* __restrict__ count, int64_t nf,
                                                 int k, int max_iter, int chunk,
                                                 float* __restrict__ params,
                                                 int32_t* __restrict__ iters,
                                                 int32_t* __restrict__ status,
                                                 float* __restrict__ chi2_out, int status_code) {
  const int lane = lane_id();
  const int grp = lane >> 4;
  const int gl = lane & 15;
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
  int64_t next = base + 4;  // wave-uniform hand-out index
  bool active = s < end;
  bool fresh = true;
  float yv[Q];
  double c = 0, w = 1, d = 0, b = 0, lam = 1e-3;
  int it = 0;
  int64_t fi = 0;  // frame of the current spectrum
  Sums cur;
  if (active) {
    fi = idx ? (int64_t)idx[s] : s;
    load_spectrum<Q>(y, fi, k, yv);
    c = p0[fi * 4 + 0];
    w = p0[fi * 4 + 1];
    d = p0[fi * 4 + 2];
    b = p0[fi * 4 + 3];
  } else {
#pragma unroll
    for (int q = 0; q < Q; ++q) yv[q] = 0.0f;
  }

  while (__ballot(active) != 0ull) {
    // 1. damped step for groups past their start point
    double delta[4] = {0.0, 0.0, 0.0, 0.0};
    bool solved = false;
    if (active && !fresh) solved = damped_solve(cur, lam, delta);
    const double tc = c + delta[0], tw = w + delta[1], td = d + delta[2], tb = b + delta[3];
    const bool point_ok = fresh || (solved && isfinite(tc) && isfinite(tw) && isfinite(td) &&
                                    isfinite(tb) && tw > 0.0);
    // 2. evaluation (start point for fresh groups, trial point otherwise)
    Sums trial;
    evaluate<Q>(yv, k, active && point_ok, tc, tw, td, tb, trial);
    // 3. decisions
    bool done = false;
    int st = CG_FIT_MAX_ITER;
    if (active) {
      if (fresh) {
        fresh = false;
        cur = trial;
        it = 0;
        lam = 1e-3;
        if (!isfinite(cur.chi2)) {
          done = true;
          st = CG_FIT_SINGULAR;
        } else if (cur.chi2 <= 1e-30) {
          done = true;
          st = CG_FIT_CONVERGED;
        }
      } else {
        ++it;
        if (!solved) {
          done = true;
          st = CG_FIT_SINGULAR;
        } else if (point_ok && isfinite(trial.chi2) && trial.chi2 <= cur.chi2) {
          const double old = cur.chi2;
          const double drop = old - trial.chi2;
          c = tc;
          w = tw;
          d = td;
          b = tb;
          cur = trial;
          lam *= 0.1;
          if (drop <= 1e-6 * old || cur.chi2 <= 1e-30) {
            done = true;
            st = CG_FIT_CONVERGED;
          }
        } else {
          lam *= 10.0;
        }
        if (!done && it >= max_iter) {
          done = true;
          st = CG_FIT_MAX_ITER;
        }
      }
    }
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
        const uint64_t below = fin & ((1ull << (grp * 16)) - 1ull);
        s = next + __popcll(below);
        active = s < end;
        fresh = true;
        if (active) {
          fi = idx ? (int64_t)idx[s] : s;
          load_spectrum<Q>(y, fi, k, yv);
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

__global__ void zero_i32_kernel(int32_t* p) { *p = 0; }

__global__ void fallback_select_kernel(const float* __restrict__ chi2, int64_t nf, int k,
                                       float thr2, int32_t* __restrict__ flags,
                                       int32_t* __restrict__ idx, int32_t* __restrict__ count,
                                       const int32_t* __restrict__ dev_n) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (dev_n) {
    const int64_t dn = *dev_n;
    nf = dn < nf ? dn : nf;
  }
  if (f >= nf) return;
  // RMS residual sqrt(chi2 / (k - 4)) > 2 sigma  <=>  chi2 > 4 sigma^2 (k - 4)
  const float c = chi2[f];
  const bool bad = !isfinite(c) || c > thr2;
  flags[f] = bad ? 1 : 0;
  if (bad) idx[atomicAdd(count, 1)] = (int32_t)f;
}

}  // namespace

hipError_t launch_fallback_select(const float* chi2, int64_t nf, int k, float noise_floor,
                                  int32_t* flags, int32_t* idx, int32_t* count, hipStream_t s,
                                  const int32_t* dev_n) {
  hipLaunchKernelGGL(zero_i32_kernel, dim3(1), dim3(1), 0, s, count);
  const double dof = k > 4 ? (double)(k - 4) : 1.0;
  const float thr2 = (float)(4.0 * (double)noise_floor * (double)noise_floor * dof);
  const int64_t blocks = (nf + 255) / 256;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fallback_select_kernel, dim3((unsigned)blocks), dim3(256), 0, s, chi2, nf, k,
                     thr2, flags, idx, count, dev_n);
  return hipGetLastError();
}

int lm_chunk(int64_t nf) {
  // spectra per wave: enough waves to fill 256 CUs several times over, and at
  // least a few spectra per group so finished groups have work to take
  int64_t c = (nf + 8191) / 8192;
  c = ((c + 3) / 4) * 4;
  if (c < 4) c = 4;
  if (c > 64) c = 64;
  return (int)c;
}

hipError_t launch_lm(const float* y, const float* p0, int64_t nf, int k, int max_iter,
                     float* params, int32_t* iters, int32_t* status, float* chi2, hipStream_t s,
                     int chunk, const int32_t* dev_n) {
  if (chunk <= 0) chunk = lm_chunk(nf);
  const int64_t waves = (nf + chunk - 1) / chunk;
  const int64_t blocks = (waves + 3) / 4;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  CG_DISPATCH_Q16(k, hipLaunchKernelGGL(lm_kernel<Q>, dim3((unsigned)blocks), dim3(256), 0, s, y,
                                        p0, nullptr, dev_n, nf, k, max_iter, chunk, params,
                                        iters, status, chi2, -1));
  return hipGetLastError();
}

hipError_t launch_lm_indexed(const float* y, const float* p0, const int32_t* idx,
                             const int32_t* count, int64_t n_cap, int k, int max_iter,
                             float* params, int32_t* iters, int32_t* status, float* chi2,
                             int32_t status_code, hipStream_t s) {
  const int chunk = 4;  // the count is only known on the device: small chunks keep waves busy
  const int64_t waves = (n_cap + chunk - 1) / chunk;
  const int64_t blocks = (waves + 3) / 4;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  CG_DISPATCH_Q16(k, hipLaunchKernelGGL(lm_kernel<Q>, dim3((unsigned)blocks), dim3(256), 0, s, y,
                                        p0, idx, count, n_cap, k, max_iter, chunk, params, iters,
                                        status, chi2, status_code));
  return hipGetLastError();
}

}  // namespace cg
