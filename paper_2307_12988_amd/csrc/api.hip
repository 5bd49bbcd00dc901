// Host side of the C ABI declared in include/combgpu.h: argument validation
// (before any HIP call), plan lifetime, workspace and kernel sequencing.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <unordered_set>

#include "internal.h"
#include "mlp.h"

namespace cg {

namespace {
thread_local std::string g_detail;

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

size_t image_bytes(int64_t nf, int k) { return align256((size_t)nf * (size_t)k * sizeof(float)); }

// workspace layout: y image | start points [nf][4] | chi2 [nf] | fallback
// flags [nf] | fallback list [nf] | fallback count
size_t ws_bytes(int64_t nf, int k) {
  return image_bytes(nf, k) + align256((size_t)nf * 4 * sizeof(float)) +
         3 * align256((size_t)nf * sizeof(float)) + 256;
}

bool is_pow2(int32_t v) { return v > 0 && (v & (v - 1)) == 0; }

cg_status check_geometry(int32_t n, double fs, const int32_t* bins, int32_t k,
                         int32_t sample_type) {
  if (!bins) return CG_ERR_NULL;
  if (sample_type != CG_SAMPLES_INT16 && sample_type != CG_SAMPLES_INT8) {
    set_detail("sample_type must be CG_SAMPLES_INT16 or CG_SAMPLES_INT8");
    return CG_ERR_INVALID_ARG;
  }
  const bool pow2 = is_pow2(n) && n >= CG_MIN_FRAME_LEN && n <= CG_MAX_FRAME_LEN;
  if (n != CG_PAPER_FRAME_LEN && !(pow2 && sample_type == CG_SAMPLES_INT16)) {
    set_detail("frame_len must be a power of two in [512, 8192] (int16 samples) or 2200 "
               "(int8 or int16 samples)");
    return CG_ERR_UNSUPPORTED;
  }
  if (k < 1) {
    set_detail("n_teeth must be >= 1");
    return CG_ERR_INVALID_ARG;
  }
  if (k > CG_MAX_TEETH || k > n / 2 + 1) {
    set_detail("n_teeth exceeds min(440, frame_len/2+1)");
    return CG_ERR_UNSUPPORTED;
  }
  if (!(fs > 0.0) || !std::isfinite(fs)) {
    set_detail("fs must be finite and > 0");
    return CG_ERR_INVALID_ARG;
  }
  std::unordered_set<int32_t> seen;
  for (int32_t i = 0; i < k; ++i) {
    if (bins[i] < 0 || bins[i] > n / 2) {
      set_detail("tooth bin outside [0, frame_len/2]");
      return CG_ERR_INVALID_ARG;
    }
    if (!seen.insert(bins[i]).second) {
      set_detail("duplicate tooth bin");
      return CG_ERR_INVALID_ARG;
    }
  }
  return CG_OK;
}

cg_status check_ref(const float* ref, int32_t k) {
  if (!ref) return CG_ERR_NULL;
  for (int32_t i = 0; i < k; ++i) {
    if (!std::isfinite(ref[i]) || !(ref[i] > 0.0f)) {
      set_detail("reference spectrum must be finite and > 0");
      return CG_ERR_BAD_REF;
    }
  }
  return CG_OK;
}

hipStream_t pick(const cg_plan*, void* s) { return reinterpret_cast<hipStream_t>(s); }

bool aligned(const void* ptr, size_t a) { return (reinterpret_cast<uintptr_t>(ptr) % a) == 0; }

}  // namespace

// reference and 0.5/reference (the FFT epilogue multiplies 2|X| by it)
hipError_t upload_reference(cg_plan* p, const float* ref) {
  std::vector<float> half_inv(p->k);
  for (int i = 0; i < p->k; ++i) half_inv[i] = (float)(0.5 / (double)ref[i]);
  hipError_t e = hipMemcpy(p->d_ref, ref, sizeof(float) * p->k, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(p->d_half_inv_ref, half_inv.data(), sizeof(float) * p->k,
                  hipMemcpyHostToDevice);
  return e;
}

namespace {

// Grow the plan-owned workspace to at least `bytes`.
cg_status ensure_ws(cg_plan* p, size_t bytes) {
  if (bytes <= p->ws_bytes) return CG_OK;
  hipError_t e = hipDeviceSynchronize();  // the old buffer may still be in use
  if (e != hipSuccess) return hip_fail(e, "workspace grow: sync");
  if (p->ws) (void)hipFree(p->ws);
  p->ws = nullptr;
  p->ws_bytes = 0;
  e = hipMalloc(&p->ws, bytes);
  if (e != hipSuccess) return hip_fail(e, "workspace grow: hipMalloc");
  p->ws_bytes = bytes;
  return CG_OK;
}

void free_plan(cg_plan* p) {
  if (!p) return;
  (void)hipDeviceSynchronize();
  if (p->d_bins) (void)hipFree(p->d_bins);
  if (p->d_ref) (void)hipFree(p->d_ref);
  if (p->d_half_inv_ref) (void)hipFree(p->d_half_inv_ref);
  if (p->d_tw) (void)hipFree(p->d_tw);
  if (p->d_tw_mixed) (void)hipFree(p->d_tw_mixed);
  if (p->d_tooth_w) (void)hipFree(p->d_tooth_w);
  if (p->d_mx_list) (void)hipFree(p->d_mx_list);
  if (p->ws) (void)hipFree(p->ws);
  for (auto* b : p->d_mfma_bf)
    if (b) (void)hipFree(b);
  for (auto* b : p->d_mfma_h)
    if (b) (void)hipFree(b);
  free_mlp(p->mlp);
  delete p;
}

}  // namespace

void set_detail(const std::string& s) { g_detail = s; }

cg_status hip_fail(hipError_t e, const char* where) {
  set_detail(std::string(where) + ": " + hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? CG_ERR_OOM : CG_ERR_HIP;
}

}  // namespace cg

using cg::hip_fail;

extern "C" {

const char* cg_status_string(cg_status s) {
  switch (s) {
    case CG_OK: return "ok";
    case CG_ERR_INVALID_ARG: return "invalid argument";
    case CG_ERR_UNSUPPORTED: return "unsupported frame length or tooth count";
    case CG_ERR_BAD_REF: return "reference spectrum must be finite and > 0";
    case CG_ERR_NULL: return "required pointer is NULL";
    case CG_ERR_OOM: return "device allocation failed";
    case CG_ERR_HIP: return "HIP runtime error";
    case CG_ERR_WORKSPACE: return "workspace too small";
    case CG_ERR_STATE: return "plan lacks the state this operation needs";
    case CG_ERR_RING_FULL: return "ring full: burst not taken (overflow)";
    default: return "unknown status";
  }
}

const char* cg_last_error_detail(void) { return cg::g_detail.c_str(); }

const char* cg_version(void) { return "combgpu-mi355x 0.1.0 gfx950"; }

cg_status cg_create_plan(int32_t frame_len, double fs, const int32_t* tooth_bins,
                         int32_t n_teeth, const float* ref_spectrum, cg_plan** out_plan) {
  return cg_create_plan_ex(frame_len, fs, tooth_bins, n_teeth, ref_spectrum, CG_SAMPLES_INT16,
                           out_plan);
}

cg_status cg_create_plan_ex(int32_t frame_len, double fs, const int32_t* tooth_bins,
                            int32_t n_teeth, const float* ref_spectrum, int32_t sample_type,
                            cg_plan** out_plan) {
  cg::set_detail("");
  if (!out_plan) return CG_ERR_NULL;
  *out_plan = nullptr;
  cg_status st = cg::check_geometry(frame_len, fs, tooth_bins, n_teeth, sample_type);
  if (st != CG_OK) return st;
  st = cg::check_ref(ref_spectrum, n_teeth);
  if (st != CG_OK) return st;

  cg_plan* p = new (std::nothrow) cg_plan();
  if (!p) return CG_ERR_OOM;
  p->n = frame_len;
  p->m = frame_len / 2;
  p->sample_bytes = sample_type == CG_SAMPLES_INT8 ? 1 : 2;
  p->k = n_teeth;
  p->fs = fs;
  p->h_bins.assign(tooth_bins, tooth_bins + n_teeth);
  p->h_ref.assign(ref_spectrum, ref_spectrum + n_teeth);

  // twiddles W_N^e built in FP64 and rounded once
  std::vector<float2> tw(frame_len);
  for (int32_t e = 0; e < frame_len; ++e) {
    const double a = 2.0 * (double)e / (double)frame_len;  // angle / pi, exact
    tw[e].x = (float)std::cos(M_PI * a);
    tw[e].y = (float)-std::sin(M_PI * a);
  }
  hipError_t e;
#define CG_TRY(call, what)                 \
  do {                                      \
    e = (call);                             \
    if (e != hipSuccess) {                  \
      st = hip_fail(e, what);               \
      cg::free_plan(p);                     \
      return st;                            \
    }                                       \
  } while (0)
  CG_TRY(hipGetDevice(&p->device), "hipGetDevice");
  CG_TRY(hipMalloc(&p->d_bins, sizeof(int32_t) * n_teeth), "hipMalloc bins");
  CG_TRY(hipMalloc(&p->d_ref, sizeof(float) * n_teeth), "hipMalloc ref");
  CG_TRY(hipMalloc(&p->d_half_inv_ref, sizeof(float) * n_teeth), "hipMalloc inverse ref");
  CG_TRY(hipMalloc(&p->d_tw, sizeof(float2) * frame_len), "hipMalloc twiddles");
  CG_TRY(hipMemcpy(p->d_bins, tooth_bins, sizeof(int32_t) * n_teeth, hipMemcpyHostToDevice),
         "copy bins");
  CG_TRY(cg::upload_reference(p, ref_spectrum), "copy ref");
  CG_TRY(hipMemcpy(p->d_tw, tw.data(), sizeof(float2) * frame_len, hipMemcpyHostToDevice),
         "copy twiddles");
  if (frame_len == CG_PAPER_FRAME_LEN) {
    // mixed-radix tables: W_M^e of the 1100-point complex FFT and, per
    // tooth, W_N^bin of the real-FFT untangling, built in FP64
    const int32_t m = frame_len / 2;
    std::vector<float2> twm(m), ttw(n_teeth);
    for (int32_t e = 0; e < m; ++e) {
      const double a = 2.0 * (double)e / (double)m;
      twm[e].x = (float)std::cos(M_PI * a);
      twm[e].y = (float)-std::sin(M_PI * a);
    }
    for (int32_t i = 0; i < n_teeth; ++i) {
      const double a = 2.0 * (double)tooth_bins[i] / (double)frame_len;
      ttw[i].x = (float)std::cos(M_PI * a);
      ttw[i].y = (float)-std::sin(M_PI * a);
    }
    CG_TRY(hipMalloc(&p->d_tw_mixed, sizeof(float2) * m), "hipMalloc mixed twiddles");
    CG_TRY(hipMalloc(&p->d_tooth_w, sizeof(float2) * n_teeth), "hipMalloc tooth twiddles");
    CG_TRY(hipMemcpy(p->d_tw_mixed, twm.data(), sizeof(float2) * m, hipMemcpyHostToDevice),
           "copy mixed twiddles");
    CG_TRY(hipMemcpy(p->d_tooth_w, ttw.data(), sizeof(float2) * n_teeth, hipMemcpyHostToDevice),
           "copy tooth twiddles");
    CG_TRY(cg::mixed_prepare(p), "mixed-radix butterfly lists");
  }
  CG_TRY(cg::resolve_static_scratch(p->device), "fixed scratch: hipGetSymbolAddress");
#undef CG_TRY
  p->fft_blocks = cg::fft_grid_limit(p);
  {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) ==
            hipSuccess &&
        cus > 0)
      cg::set_compute_units(cus);
  }
  *out_plan = p;
  return CG_OK;
}

cg_status cg_destroy_plan(cg_plan* p) {
  cg::free_plan(p);
  return CG_OK;
}

cg_status cg_set_reference(cg_plan* p, const float* ref) {
  if (!p) return CG_ERR_NULL;
  cg_status st = cg::check_ref(ref, p->k);
  if (st != CG_OK) return st;
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = cg::upload_reference(p, ref);
  if (e != hipSuccess) return hip_fail(e, "cg_set_reference");
  p->h_ref.assign(ref, ref + p->k);
  return CG_OK;
}

cg_status cg_plan_sample_bytes(const cg_plan* p, int32_t* bytes) {
  if (!p || !bytes) return CG_ERR_NULL;
  *bytes = p->sample_bytes;
  return CG_OK;
}

cg_status cg_plan_info(const cg_plan* p, int32_t* frame_len, int32_t* n_teeth, double* fs) {
  if (!p) return CG_ERR_NULL;
  if (frame_len) *frame_len = p->n;
  if (n_teeth) *n_teeth = p->k;
  if (fs) *fs = p->fs;
  return CG_OK;
}

cg_status cg_workspace_bytes(const cg_plan* p, int64_t n_frames, size_t* bytes) {
  if (!p || !bytes) return CG_ERR_NULL;
  if (n_frames < 0) return CG_ERR_INVALID_ARG;
  *bytes = cg::ws_bytes(n_frames, p->k);
  return CG_OK;
}

}  // extern "C"

namespace cg {
namespace {

// The whole path of cg_process_batch_ex.  Workspace: the caller's buffer if
// given, else the fixed scratch array when no_alloc (no allocation of any
// kind, matrix-core forms refused since they build their basis on first use),
// else the plan's own, grown on demand.
cg_status process_impl(cg_plan* p, const void* frames, int64_t nf, float* out_params,
                       int32_t* out_iters, int32_t* out_status, float* out_chi2,
                       float* out_teeth, float* out_y, uint32_t flags, void* workspace,
                       size_t workspace_bytes, void* stream, bool no_alloc) {
  set_detail("");
  if (!p) return CG_ERR_NULL;
  if (nf < 0) return CG_ERR_INVALID_ARG;
  if ((flags & ~(CG_DFT_MASK | CG_FIT_MASK)) != 0u) return CG_ERR_INVALID_ARG;
  const uint32_t dft = flags & CG_DFT_MASK;
  const uint32_t fit = flags & CG_FIT_MASK;
  if (dft > CG_DFT_MFMA_FP16X2) return CG_ERR_INVALID_ARG;
  if (fit != CG_FIT_COLD && fit != CG_FIT_WARM_MLP && fit != CG_FIT_NONE && fit != CG_FIT_FANO)
    return CG_ERR_INVALID_ARG;
  if (nf == 0) return CG_OK;
  if (fit != CG_FIT_NONE && !out_params) return CG_ERR_NULL;
  if (fit == CG_FIT_NONE && !out_teeth && !out_y) return CG_ERR_NULL;
  if (!frames) return CG_ERR_NULL;
  if (!cg::aligned(frames, 4)) {
    cg::set_detail("frames must be 4-byte aligned");
    return CG_ERR_INVALID_ARG;
  }
  if (dft != CG_DFT_FFT && (p->sample_bytes != 2 || p->n == CG_PAPER_FRAME_LEN)) {
    cg::set_detail("the matrix-core forms take int16 frames of a power-of-two length");
    return CG_ERR_UNSUPPORTED;
  }
  if (dft != CG_DFT_FFT) {
    if (no_alloc) {
      cg::set_detail("the entry point that allocates nothing supports the FFT form only");
      return CG_ERR_INVALID_ARG;
    }
    if (!cg::aligned(frames, 16)) {
      cg::set_detail("matrix-core DFT forms need 16-byte aligned frames");
      return CG_ERR_INVALID_ARG;
    }
    cg_status st = cg::mfma_prepare(p, dft);
    if (st != CG_OK) return st;
  }
  if (fit == CG_FIT_WARM_MLP && !p->mlp) {
    cg::set_detail("learned warm start needs cg_set_mlp first");
    return CG_ERR_STATE;
  }
  if (fit == CG_FIT_FANO && !p->fano_set) {
    cg::set_detail("the Fano fit needs cg_set_fano first");
    return CG_ERR_STATE;
  }
  const hipStream_t s = cg::pick(p, stream);
  const size_t img = cg::image_bytes(nf, p->k);
  const size_t need = cg::ws_bytes(nf, p->k);
  char* ws;
  if (workspace) {
    if (workspace_bytes < need) return CG_ERR_WORKSPACE;
    if (!cg::aligned(workspace, 256)) {
      cg::set_detail("workspace must be 256-byte aligned");
      return CG_ERR_INVALID_ARG;
    }
    ws = static_cast<char*>(workspace);
  } else if (no_alloc) {
    if (need > (size_t)CG_STATIC_SCRATCH_BYTES) {
      cg::set_detail("batch needs " + std::to_string(need) + " bytes of scratch, more than the " +
                     std::to_string((size_t)CG_STATIC_SCRATCH_BYTES) +
                     " bytes of the fixed scratch array");
      return CG_ERR_WORKSPACE;
    }
    ws = static_cast<char*>(cg::static_scratch(p->device));
    if (!ws) {
      cg::set_detail("fixed scratch array not resolved on the plan's device");
      return CG_ERR_STATE;
    }
  } else {
    cg_status st = cg::ensure_ws(p, need);
    if (st != CG_OK) return st;
    ws = static_cast<char*>(p->ws);
  }
  float* y = out_y ? out_y : reinterpret_cast<float*>(ws);
  char* cur = ws + img;
  float* p0 = reinterpret_cast<float*>(cur);
  cur += cg::align256((size_t)nf * 4 * sizeof(float));
  float* chi2_ws = reinterpret_cast<float*>(cur);
  cur += cg::align256((size_t)nf * sizeof(float));
  int32_t* fb_flags = reinterpret_cast<int32_t*>(cur);
  cur += cg::align256((size_t)nf * sizeof(float));
  int32_t* fb_idx = reinterpret_cast<int32_t*>(cur);
  cur += cg::align256((size_t)nf * sizeof(float));
  int32_t* fb_count = reinterpret_cast<int32_t*>(cur);
  hipError_t e = dft == CG_DFT_FFT ? cg::launch_fft_teeth(p, frames, nf, out_teeth, y, s)
                                   : cg::launch_mfma_teeth(p, dft, static_cast<const int16_t*>(frames),
                                                           nf, out_teeth, y, s);
  if (e != hipSuccess) return hip_fail(e, "tooth transform launch");
  if (fit == CG_FIT_NONE) return CG_OK;
  if (fit == CG_FIT_WARM_MLP) {
    float* chi2 = out_chi2 ? out_chi2 : chi2_ws;
    e = cg::launch_mlp_infer(p->mlp, y, nf, p->k, p0, s);
    if (e == hipSuccess)
      e = cg::launch_lm(y, p0, nf, p->k, p->polish_iters, out_params, out_iters, out_status,
                        chi2, s, p->lm_chunk, nullptr, fb_count, p->lm_lanes);
    if (e == hipSuccess)
      e = cg::launch_fallback_select(chi2, nf, p->k, p->mlp->noise_floor, fb_flags, fb_idx,
                                     fb_count, s);
    if (e == hipSuccess) e = cg::launch_median_start(y, nf, p->k, nullptr, p0, s, fb_flags);
    if (e == hipSuccess)
      e = cg::launch_lm_indexed(y, p0, fb_idx, fb_count, nf, p->k, 20, out_params, out_iters,
                                out_status, chi2, CG_FIT_FALLBACK, s);
    if (e != hipSuccess) return hip_fail(e, "warm-start launch");
    return CG_OK;
  }
  // the Fano fit starts from the median centre alone
  e = cg::launch_median_start(y, nf, p->k, nullptr, p0, s, nullptr, nullptr,
                              fit == CG_FIT_FANO);
  if (e != hipSuccess) return hip_fail(e, "median/start launch");
  if (fit == CG_FIT_FANO) {
    e = cg::launch_fano(p, y, p0, nf, 20, out_params, out_iters, out_status, out_chi2, s);
    if (e != hipSuccess) return hip_fail(e, "fano launch");
    return CG_OK;
  }
  e = cg::launch_lm(y, p0, nf, p->k, 20, out_params, out_iters, out_status, out_chi2, s,
                    p->lm_chunk, nullptr, nullptr, p->lm_lanes);
  if (e != hipSuccess) return hip_fail(e, "lm launch");
  return CG_OK;
}

}  // namespace
}  // namespace cg

extern "C" {

cg_status cg_process_batch_ex(cg_plan* p, const void* frames, int64_t nf, float* out_params,
                              int32_t* out_iters, int32_t* out_status, float* out_chi2,
                              float* out_teeth, float* out_y, uint32_t flags, void* workspace,
                              size_t workspace_bytes, void* stream) {
  return cg::process_impl(p, frames, nf, out_params, out_iters, out_status, out_chi2, out_teeth,
                          out_y, flags, workspace, workspace_bytes, stream, false);
}

cg_status cg_process_batch_static(cg_plan* p, const void* frames, int64_t nf,
                                  float* out_params, int32_t* out_iters, int32_t* out_status,
                                  float* out_chi2, uint32_t flags, void* stream) {
  return cg::process_impl(p, frames, nf, out_params, out_iters, out_status, out_chi2, nullptr,
                          nullptr, flags, nullptr, 0, stream, true);
}

cg_status cg_process_batch(cg_plan* p, const void* frames, int64_t nf, float* out_params,
                           void* stream) {
  return cg_process_batch_ex(p, frames, nf, out_params, nullptr, nullptr, nullptr, nullptr,
                             nullptr, CG_DFT_FFT | CG_FIT_COLD, nullptr, 0, stream);
}

cg_status cg_teeth(cg_plan* p, const void* frames, int64_t nf, float* out_teeth, float* out_y,
                   uint32_t flags, void* stream) {
  if (!p) return CG_ERR_NULL;
  if ((flags & ~CG_DFT_MASK) != 0u || flags > CG_DFT_MFMA_FP16X2) return CG_ERR_INVALID_ARG;
  return cg_process_batch_ex(p, frames, nf, nullptr, nullptr, nullptr, nullptr, out_teeth, out_y,
                             flags | CG_FIT_NONE, nullptr, 0, stream);
}

cg_status cg_reference_from_frames(cg_plan* p, const void* ref_frames, int64_t n,
                                   float* out_ref, void* stream) {
  if (!p || !out_ref) return CG_ERR_NULL;
  if (n <= 0) return CG_ERR_INVALID_ARG;
  if (!ref_frames) return CG_ERR_NULL;
  if (!cg::aligned(ref_frames, 4)) return CG_ERR_INVALID_ARG;
  const hipStream_t s = cg::pick(p, stream);
  float* mags = nullptr;
  hipError_t e = hipMalloc(&mags, (size_t)n * p->k * sizeof(float));
  if (e != hipSuccess) return hip_fail(e, "reference: hipMalloc");
  e = cg::launch_fft_teeth(p, ref_frames, n, mags, nullptr, s);
  if (e == hipSuccess) e = cg::launch_column_mean(mags, n, p->k, out_ref, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(mags);
  if (e != hipSuccess) return hip_fail(e, "reference");
  return CG_OK;
}

cg_status cg_init_spectra(cg_plan* p, const float* y, int64_t nf, float* out_p0, float* out_median,
                          void* stream) {
  if (!p || !out_p0) return CG_ERR_NULL;
  if (nf < 0) return CG_ERR_INVALID_ARG;
  if (nf == 0) return CG_OK;
  if (!y) return CG_ERR_NULL;
  if (y == out_median) return CG_ERR_INVALID_ARG;
  hipError_t e = cg::launch_median_start(y, nf, p->k, out_median, out_p0, cg::pick(p, stream));
  if (e != hipSuccess) return hip_fail(e, "init launch");
  return CG_OK;
}

cg_status cg_start_centres(cg_plan* p, const float* y, int64_t nf, float* out_p0, void* stream) {
  if (!p || !out_p0) return CG_ERR_NULL;
  if (nf < 0) return CG_ERR_INVALID_ARG;
  if (nf == 0) return CG_OK;
  if (!y) return CG_ERR_NULL;
  hipError_t e = cg::launch_median_start(y, nf, p->k, nullptr, out_p0, cg::pick(p, stream),
                                         nullptr, nullptr, true);
  if (e != hipSuccess) return hip_fail(e, "start centres launch");
  return CG_OK;
}

cg_status cg_init_spectra_listed(cg_plan* p, const float* y, int64_t nf, const int32_t* listed,
                                 float* out_p0, void* stream) {
  if (!p || !out_p0) return CG_ERR_NULL;
  if (nf < 0) return CG_ERR_INVALID_ARG;
  if (nf == 0) return CG_OK;
  if (!y || !listed) return CG_ERR_NULL;
  hipError_t e =
      cg::launch_median_start(y, nf, p->k, nullptr, out_p0, cg::pick(p, stream), listed);
  if (e != hipSuccess) return hip_fail(e, "listed init launch");
  return CG_OK;
}

cg_status cg_median_filter(cg_plan* p, const float* y, int64_t nf, float* out_median,
                           void* stream) {
  if (!p || !out_median) return CG_ERR_NULL;
  if (nf < 0) return CG_ERR_INVALID_ARG;
  if (nf == 0) return CG_OK;
  if (!y) return CG_ERR_NULL;
  if (y == out_median) return CG_ERR_INVALID_ARG;
  hipError_t e = cg::launch_median_start(y, nf, p->k, out_median, nullptr, cg::pick(p, stream));
  if (e != hipSuccess) return hip_fail(e, "median launch");
  return CG_OK;
}

cg_status cg_start_points(cg_plan* p, const float* median, int64_t nf, float* out_p0,
                          void* stream) {
  if (!p || !out_p0) return CG_ERR_NULL;
  if (nf < 0) return CG_ERR_INVALID_ARG;
  if (nf == 0) return CG_OK;
  if (!median) return CG_ERR_NULL;
  hipError_t e = cg::launch_start_points(median, nf, p->k, out_p0, cg::pick(p, stream));
  if (e != hipSuccess) return hip_fail(e, "start point launch");
  return CG_OK;
}

cg_status cg_fit_spectra(cg_plan* p, const float* y, const float* p0, int64_t nf, int32_t max_iter,
                         float* out_params, int32_t* out_iters, int32_t* out_status,
                         float* out_chi2, void* stream) {
  if (!p || !out_params) return CG_ERR_NULL;
  if (nf < 0 || max_iter < 1 || max_iter > CG_MAX_ITER) return CG_ERR_INVALID_ARG;
  if (nf == 0) return CG_OK;
  if (!y || !p0) return CG_ERR_NULL;
  const hipStream_t s = cg::pick(p, stream);
  hipError_t e = cg::launch_lm(y, p0, nf, p->k, max_iter, out_params, out_iters, out_status,
                               out_chi2, s, p->lm_chunk, nullptr, nullptr, p->lm_lanes);
  if (e != hipSuccess) return hip_fail(e, "lm launch");
  return CG_OK;
}

cg_status cg_set_fano(cg_plan* p, double width, double asymmetry, double depth_avg,
                      double scale_avg) {
  if (!p) return CG_ERR_NULL;
  if (!std::isfinite(width) || !(width > 0.0) || !std::isfinite(asymmetry) ||
      !(std::fabs(asymmetry) >= 1e-3) || !std::isfinite(depth_avg) || !(depth_avg > 0.0) ||
      !std::isfinite(scale_avg) || !(scale_avg > 0.0)) {
    cg::set_detail("width > 0, |asymmetry| >= 1e-3 and averages > 0, all finite");
    return CG_ERR_INVALID_ARG;
  }
  p->fano_w = width;
  p->fano_q = asymmetry;
  p->fano_dbar = depth_avg;
  p->fano_bbar = scale_avg;
  p->fano_set = true;
  return CG_OK;
}

cg_status cg_fit_fano(cg_plan* p, const float* y, const float* p0, int64_t nf, int32_t max_iter,
                      float* out_params, int32_t* out_iters, int32_t* out_status,
                      float* out_chi2, void* stream) {
  if (!p || !out_params) return CG_ERR_NULL;
  if (nf < 0 || max_iter < 1 || max_iter > CG_MAX_ITER) return CG_ERR_INVALID_ARG;
  if (!p->fano_set) {
    cg::set_detail("the Fano fit needs cg_set_fano first");
    return CG_ERR_STATE;
  }
  if (nf == 0) return CG_OK;
  if (!y || !p0) return CG_ERR_NULL;
  hipError_t e = cg::launch_fano(p, y, p0, nf, max_iter, out_params, out_iters, out_status,
                                 out_chi2, cg::pick(p, stream));
  if (e != hipSuccess) return hip_fail(e, "fano launch");
  return CG_OK;
}

namespace {
bool psd_len_ok(int32_t seg_len) {
  return seg_len == 16384 || seg_len == 32768 || seg_len == 65536 || seg_len == 131072;
}
int64_t psd_segments(int64_t n, int32_t seg_len) {
  return n < seg_len ? 0 : (n - seg_len) / (seg_len / 2) + 1;
}
int64_t psd_chunk(int64_t n_seg) { return n_seg < CG_PSD_CHUNK ? n_seg : CG_PSD_CHUNK; }
}  // namespace

cg_status cg_psd_band(int32_t seg_len, double fs, double f_lo, double f_hi, int32_t* k_lo,
                      int32_t* n_bins) {
  if (!k_lo || !n_bins) return CG_ERR_NULL;
  if (!psd_len_ok(seg_len) || !(fs > 0.0) || !std::isfinite(fs) || !std::isfinite(f_lo) ||
      !std::isfinite(f_hi) || !(f_lo >= 0.0) || !(f_hi >= f_lo))
    return CG_ERR_INVALID_ARG;
  const double bin = fs / (double)seg_len;
  int64_t lo = (int64_t)std::ceil(f_lo / bin), hi = (int64_t)std::floor(f_hi / bin);
  if (hi > seg_len / 2) hi = seg_len / 2;
  if (hi < lo) return CG_ERR_INVALID_ARG;
  *k_lo = (int32_t)lo;
  *n_bins = (int32_t)(hi - lo + 1);
  return CG_OK;
}

cg_status cg_psd_workspace_bytes(int64_t n, int32_t seg_len, int32_t n_bins, size_t* bytes) {
  if (!bytes) return CG_ERR_NULL;
  if (!psd_len_ok(seg_len) || n_bins < 1 || n < seg_len) return CG_ERR_INVALID_ARG;
  *bytes = cg::psd_workspace_bytes(psd_chunk(psd_segments(n, seg_len)), seg_len, n_bins);
  return CG_OK;
}

cg_status cg_psd_welch(const float* series, int64_t n, double fs, int32_t seg_len, int32_t k_lo,
                       int32_t n_bins, double* out_psd, void* workspace, size_t workspace_bytes,
                       void* stream) {
  cg::set_detail("");
  if (!series || !out_psd || !workspace) return CG_ERR_NULL;
  if (!psd_len_ok(seg_len) || n < seg_len || !(fs > 0.0) || !std::isfinite(fs) || k_lo < 0 ||
      n_bins < 1 || k_lo + n_bins - 1 > seg_len / 2) {
    cg::set_detail("seg_len in {2^14..2^17}, n >= seg_len, band inside [0, seg_len/2]");
    return CG_ERR_INVALID_ARG;
  }
  if (!cg::aligned(series, 8) || !cg::aligned(workspace, 256)) {
    cg::set_detail("series must be 8-byte and workspace 256-byte aligned");
    return CG_ERR_INVALID_ARG;
  }
  const int64_t chunk = psd_chunk(psd_segments(n, seg_len));
  if (workspace_bytes < cg::psd_workspace_bytes(chunk, seg_len, n_bins)) return CG_ERR_WORKSPACE;
  hipError_t e = cg::launch_psd(series, n, fs, seg_len, k_lo, n_bins, out_psd, workspace, chunk,
                                reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "psd launch");
  return CG_OK;
}

cg_status cg_resonance_fit(const double* psd, int32_t n_bins, double f_first, double df,
                           int32_t max_iter, double tol, double* out, void* stream) {
  if (!psd || !out) return CG_ERR_NULL;
  if (n_bins < 8 || n_bins > CG_PSD_MAX_FIT_BINS || !(df > 0.0) || !std::isfinite(df) ||
      !std::isfinite(f_first) || !(f_first >= 0.0) || max_iter < 1 || max_iter > 10000 ||
      !(tol >= 0.0))
    return CG_ERR_INVALID_ARG;
  hipError_t e = cg::launch_osc_fit(psd, n_bins, f_first, df, max_iter, tol, out,
                                    reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "resonance fit launch");
  return CG_OK;
}

cg_status cg_set_mlp(cg_plan* p, const float* params, const float* out_mean, const float* out_std,
                     float noise_floor) {
  if (!p || !params || !out_mean || !out_std) return CG_ERR_NULL;
  for (int i = 0; i < CG_MLP_NPARAMS; ++i)
    if (!std::isfinite(params[i])) {
      cg::set_detail("network parameters must be finite");
      return CG_ERR_INVALID_ARG;
    }
  for (int j = 0; j < 4; ++j)
    if (!std::isfinite(out_mean[j]) || !std::isfinite(out_std[j]) || !(out_std[j] > 0.f)) {
      cg::set_detail("output mean must be finite and std finite and > 0");
      return CG_ERR_INVALID_ARG;
    }
  if (!std::isfinite(noise_floor) || !(noise_floor > 0.f)) {
    cg::set_detail("noise_floor must be finite and > 0");
    return CG_ERR_INVALID_ARG;
  }
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "cg_set_mlp sync");
  cg_mlp* m = nullptr;
  cg_status st = cg::make_mlp(params, out_mean, out_std, noise_floor, &m);
  if (st != CG_OK) return st;
  cg::free_mlp(p->mlp);
  p->mlp = m;
  return CG_OK;
}

cg_status cg_mlp_infer(cg_plan* p, const float* y, int64_t nf, float* out_p0, void* stream) {
  if (!p || !out_p0) return CG_ERR_NULL;
  if (nf < 0) return CG_ERR_INVALID_ARG;
  if (!p->mlp) return CG_ERR_STATE;
  if (nf == 0) return CG_OK;
  if (!y) return CG_ERR_NULL;
  hipError_t e = cg::launch_mlp_infer(p->mlp, y, nf, p->k, out_p0, cg::pick(p, stream));
  if (e != hipSuccess) return hip_fail(e, "mlp launch");
  return CG_OK;
}

cg_status cg_mlp_trainer_create(int32_t batch, const float* init, cg_mlp_trainer** out) {
  if (!out) return CG_ERR_NULL;
  *out = nullptr;
  if (!init) return CG_ERR_NULL;
  if (batch < 1 || batch > 65536) return CG_ERR_INVALID_ARG;
  for (int i = 0; i < CG_MLP_NPARAMS; ++i)
    if (!std::isfinite(init[i])) return CG_ERR_INVALID_ARG;
  return cg::make_trainer(batch, init, out);
}

cg_status cg_mlp_trainer_destroy(cg_mlp_trainer* t) {
  cg::free_trainer(t);
  return CG_OK;
}

cg_status cg_mlp_train_step(cg_mlp_trainer* t, const float* x, const float* targets,
                            const float* weights, const int32_t* idx, float lr, float beta1,
                            float beta2, float eps, float* loss, void* stream) {
  if (!t || !x || !targets || !idx) return CG_ERR_NULL;
  if (!(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) ||
      !(eps > 0.f))
    return CG_ERR_INVALID_ARG;
  return cg::trainer_step(t, x, targets, weights, idx, lr, beta1, beta2, eps, 1, nullptr, loss,
                          reinterpret_cast<hipStream_t>(stream));
}

cg_status cg_mlp_gradients(cg_mlp_trainer* t, const float* x, const float* targets,
                           const float* weights, const int32_t* idx, float* grads, float* loss,
                           void* stream) {
  if (!t || !x || !targets || !idx || !grads) return CG_ERR_NULL;
  return cg::trainer_step(t, x, targets, weights, idx, 1.f, 0.f, 0.f, 1.f, 0, grads, loss,
                          reinterpret_cast<hipStream_t>(stream));
}

cg_status cg_mlp_get_params(cg_mlp_trainer* t, float* params) {
  if (!t || !params) return CG_ERR_NULL;
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess)
    e = hipMemcpy(params, t->params, sizeof(float) * CG_MLP_NPARAMS, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "cg_mlp_get_params");
  return CG_OK;
}

cg_status cg_set_polish_iters(cg_plan* p, int32_t iters) {
  if (!p) return CG_ERR_NULL;
  if (iters < 1 || iters > CG_MAX_ITER) return CG_ERR_INVALID_ARG;
  p->polish_iters = iters;
  return CG_OK;
}

cg_status cg_get_tuning(const cg_plan* p, int32_t knob, int32_t* value) {
  if (!p || !value) return CG_ERR_NULL;
  switch (knob) {
    case CG_TUNE_LM_CHUNK: *value = p->lm_chunk; return CG_OK;
    case CG_TUNE_LM_LANES: *value = p->lm_lanes; return CG_OK;
    case CG_TUNE_FFT_BLOCKS: *value = p->fft_cap; return CG_OK;
    default: return CG_ERR_INVALID_ARG;
  }
}

cg_status cg_set_tuning(cg_plan* p, int32_t knob, int32_t value) {
  if (!p) return CG_ERR_NULL;
  switch (knob) {
    case CG_TUNE_LM_CHUNK:
      if (value != 0 && (value < 4 || value > 256 || value % 4 != 0)) return CG_ERR_INVALID_ARG;
      p->lm_chunk = value;
      return CG_OK;
    case CG_TUNE_LM_LANES:
      if (value != 0 && value != 8 && value != 16) return CG_ERR_INVALID_ARG;
      if (value == 8 && p->k > 224) return CG_ERR_INVALID_ARG;
      p->lm_lanes = value;
      return CG_OK;
    case CG_TUNE_FFT_BLOCKS:
      if (value < 0) return CG_ERR_INVALID_ARG;
      p->fft_cap = value;
      return CG_OK;
    default:
      return CG_ERR_INVALID_ARG;
  }
}

}  // extern "C"
