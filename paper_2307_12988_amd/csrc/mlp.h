// Learned warm-start network: shapes, parameter layout and device state.
#pragma once

#include "internal.h"

namespace cg {

constexpr int MLP_IN = 220, MLP_IN_PAD = 224, MLP_HID = 256, MLP_OUT = 4;
// flat parameter layout: W1[256][220], b1[256], W2[256][256], b2[256], W3[4][256], b3[4]
constexpr int MLP_OFF_W1 = 0;
constexpr int MLP_OFF_B1 = MLP_OFF_W1 + MLP_HID * MLP_IN;
constexpr int MLP_OFF_W2 = MLP_OFF_B1 + MLP_HID;
constexpr int MLP_OFF_B2 = MLP_OFF_W2 + MLP_HID * MLP_HID;
constexpr int MLP_OFF_W3 = MLP_OFF_B2 + MLP_HID;
constexpr int MLP_OFF_B3 = MLP_OFF_W3 + MLP_OUT * MLP_HID;
constexpr int MLP_NPARAMS = MLP_OFF_B3 + MLP_OUT;
static_assert(MLP_NPARAMS == CG_MLP_NPARAMS, "parameter count");

struct MlpScale {
  float mean[4];  // output de-standardisation: p = z * std + mean
  float std[4];
};

cg_status make_mlp(const float* params, const float* mean, const float* stdv, float noise_floor,
                   cg_mlp** out);
void free_mlp(cg_mlp* m);
hipError_t launch_mlp_infer(const cg_mlp* m, const float* y, int64_t nf, int k, float* p0,
                            hipStream_t s, const int32_t* dev_n = nullptr);

cg_status make_trainer(int32_t batch, const float* init, cg_mlp_trainer** out);
void free_trainer(cg_mlp_trainer* t);
cg_status trainer_step(cg_mlp_trainer* t, const float* x, const float* tg, const float* w,
                       const int32_t* idx, float lr, float b1, float b2, float eps, int update,
                       float* grads_out, float* loss_out, hipStream_t s);

}  // namespace cg

struct cg_mlp {
  uint16_t* w1 = nullptr;  // bf16 [256][224]
  float* b1 = nullptr;     // [256]
  uint16_t* w2 = nullptr;  // bf16 [256][256]
  float* b2 = nullptr;     // [256]
  uint16_t* w3 = nullptr;  // bf16 [16][256] (rows 4..15 zero)
  float* b3 = nullptr;     // [16]
  cg::MlpScale scale{};
  float noise_floor = 0.f;
};

struct cg_mlp_trainer {
  int32_t batch = 0;
  int64_t step = 0;
  void* mem = nullptr;
  float *params = nullptr, *grads = nullptr, *m = nullptr, *v = nullptr;
  uint16_t *w1b = nullptr, *w2b = nullptr, *w3b = nullptr;
  uint16_t* xb = nullptr;
  float *tb = nullptr, *wb = nullptr;
  float* h1 = nullptr;
  uint16_t* a1b = nullptr;
  float* h2 = nullptr;
  uint16_t* a2b = nullptr;
  float *out = nullptr, *dout = nullptr;
  uint16_t* doutb = nullptr;
  float* dh2 = nullptr;
  uint16_t* dh2b = nullptr;
  float* dh1 = nullptr;
  uint16_t* dh1b = nullptr;
  float* loss = nullptr;
};
