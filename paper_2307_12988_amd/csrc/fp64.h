// FP64 reciprocal and reciprocal square root from the hardware estimates
// refined by Newton steps (shared by the fit kernels).
#pragma once

#include <hip/hip_runtime.h>

namespace cg {

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

// One Newton step on the hardware reciprocal: for arguments >= 1 (the
// per-tooth denominators) the hardware estimate is good to far more than half
// the FP64 mantissa, so one step leaves an error well below what FP64
// residuals need.
__device__ __forceinline__ double rcp1_d(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}

}  // namespace cg
