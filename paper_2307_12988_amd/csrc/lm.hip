// Batched Levenberg-Marquardt fit of the Lorentzian cavity dip, one wavefront
// per spectrum.
//
// Paper, Data Capture and Processing: each normalised spectrum is fitted by a
// Levenberg-Marquardt routine with at most 20 iterations and tolerance 1e-6;
// the fitted centre of the cavity resonance tracks the proof-mass
// displacement (Experimental Setup).  The model is the 4-parameter Lorentzian
// dip f(x) = b (1 - d / (1 + u^2)), u = 2 (x - c) / w, over tooth index x.
//
// Per iteration every lane evaluates model, residual and the four Jacobian
// columns for its teeth (i = lane + 64 q) in FP32, accumulates the 10 distinct
// entries of J^T J, the 4 of J^T r and chi2, and a butterfly all-reduce gives
// all 64 lanes bit-identical sums, so every lane takes the same decisions.
// The damped 4x4 system is solved by a Cholesky factorisation in FP64.  The
// evaluation at a trial point also yields the normal equations there, so an
// accepted step needs no second pass over the teeth.
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
  float a[10];  // J^T J upper triangle: 00 01 02 03 11 12 13 22 23 33
  float g[4];   // J^T r
  float chi2;
};

template <int Q>
__device__ __forceinline__ void evaluate(const float (&yv)[Q], int k, float c, float w, float d,
                                         float b, Sums& s) {
  const int lane = lane_id();
  float acc[15];
#pragma unroll
  for (int j = 0; j < 15; ++j) acc[j] = 0.0f;
  const float inv_w = 1.0f / w;
  const float two_iw = 2.0f * inv_w;
  const float four_iw = 4.0f * inv_w;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int i = lane + 64 * q;
    if (i < k) {
      const float u = ((float)i - c) * two_iw;
      const float den = 1.0f + u * u;
      const float id = 1.0f / den;
      const float qd = d * id;
      const float f = b * (1.0f - qd);
      const float r = yv[q] - f;
      const float t = b * qd * id;          // b d / D^2
      const float jc = -t * u * four_iw;    // -4 b d u / (w D^2)
      const float jw = -t * u * u * two_iw; // -2 b d u^2 / (w D^2)
      const float jd = -b * id;             // -b / D
      const float jb = 1.0f - qd;           // 1 - d / D
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
      acc[10] += jc * r;
      acc[11] += jw * r;
      acc[12] += jd * r;
      acc[13] += jb * r;
      acc[14] += r * r;
    }
  }
#pragma unroll
  for (int j = 0; j < 10; ++j) s.a[j] = wave_sum(acc[j]);
#pragma unroll
  for (int j = 0; j < 4; ++j) s.g[j] = wave_sum(acc[10 + j]);
  s.chi2 = wave_sum(acc[14]);
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
  const double l00 = sqrt(a00), i00 = 1.0 / l00;
  const double l10 = a01 * i00, l20 = a02 * i00, l30 = a03 * i00;
  const double t11 = a11 - l10 * l10;
  if (!(t11 > 0.0)) return false;
  const double l11 = sqrt(t11), i11 = 1.0 / l11;
  const double l21 = (a12 - l20 * l10) * i11, l31 = (a13 - l30 * l10) * i11;
  const double t22 = a22 - l20 * l20 - l21 * l21;
  if (!(t22 > 0.0)) return false;
  const double l22 = sqrt(t22), i22 = 1.0 / l22;
  const double l32 = (a23 - l30 * l20 - l31 * l21) * i22;
  const double t33 = a33 - l30 * l30 - l31 * l31 - l32 * l32;
  if (!(t33 > 0.0)) return false;
  const double l33 = sqrt(t33), i33 = 1.0 / l33;
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
__global__ __launch_bounds__(256) void lm_kernel(const float* __restrict__ y,
                                                 const float* __restrict__ m,
                                                 const float* __restrict__ p0, int64_t nf, int k,
                                                 int max_iter, float* __restrict__ params,
                                                 int32_t* __restrict__ iters,
                                                 int32_t* __restrict__ status,
                                                 float* __restrict__ chi2_out) {
  const int64_t f = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (f >= nf) return;
  const int lane = lane_id();
  float yv[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int i = lane + 64 * q;
    yv[q] = i < k ? y[f * k + i] : 0.0f;
  }
  float c, w, d, b;
  if (p0) {
    c = p0[f * 4 + 0];
    w = p0[f * 4 + 1];
    d = p0[f * 4 + 2];
    b = p0[f * 4 + 3];
  } else {
    float mv[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int i = lane + 64 * q;
      mv[q] = i < k ? m[f * k + i] : 0.0f;
    }
    start_point<Q>(mv, k, c, w, d, b);
  }

  Sums cur, trial;
  evaluate<Q>(yv, k, c, w, d, b, cur);
  int it = 0;
  int st = CG_FIT_MAX_ITER;
  if (!isfinite(cur.chi2)) {
    st = CG_FIT_SINGULAR;
  } else if (cur.chi2 <= 1e-30f) {
    st = CG_FIT_CONVERGED;
  } else {
    double lam = 1e-3;
    while (it < max_iter) {
      ++it;
      double delta[4];
      if (!damped_solve(cur, lam, delta)) {
        st = CG_FIT_SINGULAR;
        break;
      }
      const float tc = c + (float)delta[0];
      const float tw = w + (float)delta[1];
      const float td = d + (float)delta[2];
      const float tb = b + (float)delta[3];
      bool ok = isfinite(tc) && isfinite(tw) && isfinite(td) && isfinite(tb) && tw > 0.0f;
      if (ok) {
        evaluate<Q>(yv, k, tc, tw, td, tb, trial);
        ok = isfinite(trial.chi2) && trial.chi2 <= cur.chi2;
      }
      if (!ok) {
        lam *= 10.0;
        continue;
      }
      const double old = (double)cur.chi2;
      const double drop = old - (double)trial.chi2;
      c = tc;
      w = tw;
      d = td;
      b = tb;
      cur = trial;
      lam *= 0.1;
      if (drop <= 1e-6 * old || cur.chi2 <= 1e-30f) {
        st = CG_FIT_CONVERGED;
        break;
      }
    }
  }
  if (lane == 0) {
    if (params) {
      params[f * 4 + 0] = c;
      params[f * 4 + 1] = w;
      params[f * 4 + 2] = d;
      params[f * 4 + 3] = b;
    }
    if (iters) iters[f] = it;
    if (status) status[f] = st;
    if (chi2_out) chi2_out[f] = cur.chi2;
  }
}

template <int Q>
hipError_t launch_q(const float* y, const float* m, const float* p0, int64_t nf, int k,
                    int max_iter, float* params, int32_t* iters, int32_t* status, float* chi2,
                    hipStream_t s) {
  const int64_t blocks = (nf + 3) / 4;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(lm_kernel<Q>, dim3((unsigned)blocks), dim3(256), 0, s, y, m, p0, nf, k,
                     max_iter, params, iters, status, chi2);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_lm(const float* y, const float* m, const float* p0, int64_t nf, int k,
                     int max_iter, float* params, int32_t* iters, int32_t* status, float* chi2,
                     hipStream_t s) {
  switch ((k + 63) / 64) {
    case 1: return launch_q<1>(y, m, p0, nf, k, max_iter, params, iters, status, chi2, s);
    case 2: return launch_q<2>(y, m, p0, nf, k, max_iter, params, iters, status, chi2, s);
    case 3: return launch_q<3>(y, m, p0, nf, k, max_iter, params, iters, status, chi2, s);
    case 4: return launch_q<4>(y, m, p0, nf, k, max_iter, params, iters, status, chi2, s);
    case 5: return launch_q<5>(y, m, p0, nf, k, max_iter, params, iters, status, chi2, s);
    case 6: return launch_q<6>(y, m, p0, nf, k, max_iter, params, iters, status, chi2, s);
    case 7: return launch_q<7>(y, m, p0, nf, k, max_iter, params, iters, status, chi2, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace cg
