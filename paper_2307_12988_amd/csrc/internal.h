// Internal declarations shared by the library's translation units (not part of
// the public ABI; see include/combgpu.h for that).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/combgpu.h"

struct cg_mlp;  // learned warm-start weights (mlp.hip)

struct cg_plan {
  int32_t n = 0;          // frame length (samples)
  int32_t sample_bytes = 2;  // 2: int16 samples, 1: int8 samples
  int32_t m = 0;          // n / 2 : complex FFT length
  int32_t k = 0;          // number of teeth
  double fs = 0.0;        // sample rate (metadata)
  int device = 0;
  int32_t* d_bins = nullptr;   // [k] tooth bins, optical order
  float* d_ref = nullptr;      // [k] reference amplitudes
  float* d_half_inv_ref = nullptr;  // [k] 0.5 / reference (FFT epilogue)
  float2* d_tw = nullptr;      // [n] W_n^e = (cos 2 pi e/n, -sin 2 pi e/n), e = 0..n-1
  float2* d_tw_mixed = nullptr;  // 2200-sample frames: [1100] W_1100^e
  float2* d_tooth_w = nullptr;   // 2200-sample frames: [k] W_2200^bin per tooth
  // 2200-sample frames: butterflies of the last three FFT passes that the
  // teeth need, per pass 64 * mx_rounds[p] entries (-1: none), int16
  int16_t* d_mx_list = nullptr;
  int32_t mx_rounds[3] = {0, 0, 0};
  std::vector<int32_t> h_bins;
  std::vector<float> h_ref;
  void* ws = nullptr;          // plan-owned workspace (grown on demand)
  size_t ws_bytes = 0;
  cg_mlp* mlp = nullptr;
  int32_t lm_chunk = 0;        // spectra per wave in the fit kernel (0 = auto)
  int32_t lm_lanes = 0;        // lanes per spectrum in the fit kernel (0 = auto, 8, 16)
  int32_t fft_cap = 0;         // tuned cap on the FFT grid (0 = every resident block)
  int32_t polish_iters = 2;    // LM iterations from the network's start point
  // Fano fit (CG_FIT_FANO): fixed width and asymmetry, averages of extent and
  // scale (the box is +-10 % of them)
  bool fano_set = false;
  double fano_w = 0.0, fano_q = 0.0, fano_dbar = 0.0, fano_bbar = 0.0;
  int32_t fft_blocks = 0;      // resident blocks of the FFT kernel on the device (0 = no cap)
  // tooth-DFT bases for the matrix-core forms, [ceil(k/64)*64][n], built on
  // first use: bf16 cos_hi, cos_lo, sin_hi, sin_lo / fp16 cos, sin
  uint16_t* d_mfma_bf[4] = {nullptr, nullptr, nullptr, nullptr};
  uint16_t* d_mfma_h[2] = {nullptr, nullptr};
};

namespace cg {

constexpr int kWaveSize = 64;

// Copy a reference spectrum (host, k values) and its 0.5/ref table to the plan.
hipError_t upload_reference(cg_plan* p, const float* ref);

// Device address of the fixed scratch array on `device` (resolved once per
// device by resolve_static_scratch, called at plan creation; null before).
hipError_t resolve_static_scratch(int device);
void* static_scratch(int device);

// Record a HIP failure as the thread's error detail and map it to a status.
cg_status hip_fail(hipError_t e, const char* where);
void set_detail(const std::string& s);

// A1-A3: int16 frames -> raw tooth amplitudes and/or normalised spectra.
// Every launch helper takes an optional dev_n: a device int32 frame count
// read by the kernels at run time (at most n_frames, the capacity the grid is
// sized for), so one captured graph serves bursts of any size.
// Blocks of the persistent FFT kernel that fit on the plan's device at once.
// frames: n_frames x frame_len samples of the plan's sample type.
int fft_grid_limit(const cg_plan* p);
hipError_t launch_fft_teeth(const cg_plan* p, const void* frames, int64_t n_frames,
                            float* out_mag, float* out_y, hipStream_t s,
                            const int32_t* dev_n = nullptr);
// The paper's 2200-sample frames (mixed-radix FFT, int8 or int16 samples).
int fft_mixed_grid_limit(const cg_plan* p);
// Build the plan's lists of needed butterflies from its bins (host work and
// one upload; called at plan creation).
hipError_t mixed_prepare(cg_plan* p);
hipError_t launch_fft_mixed(const cg_plan* p, const void* frames, int64_t n_frames,
                            float* out_mag, float* out_y, hipStream_t s,
                            const int32_t* dev_n = nullptr);

// A6: tooth DFT on the matrix cores (form = CG_DFT_MFMA_*); mfma_prepare
// builds the plan's basis for the form on first use.
cg_status mfma_prepare(cg_plan* p, uint32_t form);
hipError_t launch_mfma_teeth(const cg_plan* p, uint32_t form, const int16_t* frames,
                             int64_t n_frames, float* out_mag, float* out_y, hipStream_t s);

// Column mean over frames of an amplitude image [n][k] -> out[k] (FP64 sums).
hipError_t launch_column_mean(const float* mags, int64_t n, int k, float* out, hipStream_t s);

// A4: 7x7 median image (out_m, may be null) and/or start points (out_p0, may
// be null) from normalised spectra, in one kernel.
// flags (may be null): only frames with flags[f] != 0 get a start point (and
// a filtered row in out_m; rows of other frames are left unwritten), and
// blocks without such frames return at once.
// centre_only: only p0[f][0] (the start centre) is written (the Fano fit's
// start; needs out_p0 and no flags or out_m: the median image is computed
// exactly only where a row's minimum can lie).
hipError_t launch_median_start(const float* y, int64_t n_frames, int k, float* out_m,
                               float* out_p0, hipStream_t s, const int32_t* flags = nullptr,
                               const int32_t* dev_n = nullptr, bool centre_only = false);
// Start points from a given median image.
hipError_t launch_start_points(const float* m, int64_t n_frames, int k, float* out_p0,
                               hipStream_t s);

// A5: Levenberg-Marquardt from start points p0.  chunk = spectra per wave
// (<= 0: chosen from n_frames and the tooth count).
// lanes = lanes per spectrum (8 or 16; 0: 8 up to 224 teeth, else 16).
int lm_group(int n_teeth);
// Compute units of the device (sizes the fit kernels' blocks; set at plan
// creation).
void set_compute_units(int cus);
// Wavefronts per block (1 .. 8) of a fit launch of `waves` wavefronts.
int fit_waves_per_block(int64_t waves);
int lm_chunk(int64_t n_frames, int n_teeth, int lanes = 0);
// zero_count, if not null, is set to 0 by the kernel (for a counter the next
// kernel on the stream accumulates into).
hipError_t launch_lm(const float* y, const float* p0, int64_t n_frames, int k, int max_iter,
                     float* params, int32_t* iters, int32_t* status, float* chi2, hipStream_t s,
                     int chunk = 0, const int32_t* dev_n = nullptr,
                     int32_t* zero_count = nullptr, int lanes = 0);
// The paper's Fano fit from the start centres p0[f][0] (plan's fixed width,
// asymmetry and box); hipErrorInvalidValue if the plan has no Fano settings.
hipError_t launch_fano(const cg_plan* p, const float* y, const float* p0, int64_t n_frames,
                       int max_iter, float* params, int32_t* iters, int32_t* status,
                       float* chi2, hipStream_t s, const int32_t* dev_n = nullptr);
// Indexed form: fit frames idx[0..*count) (count read on the device, at most
// n_cap); every reported status is replaced by status_code.
hipError_t launch_lm_indexed(const float* y, const float* p0, const int32_t* idx,
                             const int32_t* count, int64_t n_cap, int k, int max_iter,
                             float* params, int32_t* iters, int32_t* status, float* chi2,
                             int32_t status_code, hipStream_t s);
// Warm-start fallback selection: flags[f] = 1 and f appended to idx when the
// polished fit's RMS residual exceeds 2 * noise_floor or is not finite.  The
// count accumulates: it must be zero on entry (the polish launch clears it).
hipError_t launch_fallback_select(const float* chi2, int64_t n_frames, int k, float noise_floor,
                                  int32_t* flags, int32_t* idx, int32_t* count, hipStream_t s,
                                  const int32_t* dev_n = nullptr);

// Displacement PSD (Welch, band of bins) and the resonance fit (psd.hip).
size_t psd_workspace_bytes(int64_t chunk_segments, int seg_len, int n_bins);
hipError_t launch_psd(const float* x, int64_t n, double fs, int seg_len, int k_lo, int n_bins,
                      double* out, void* ws, int64_t chunk_segments, hipStream_t s);
hipError_t launch_osc_fit(const double* psd, int n_bins, double f_first, double df,
                          int max_iter, double tol, double* out, hipStream_t s);

}  // namespace cg
