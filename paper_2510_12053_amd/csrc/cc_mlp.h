// Warm-start network: sizes, packed parameter layout and device state.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cc_kernels.h"

namespace cc {

constexpr int MLP_IN = 16;      // features per vertex
constexpr int MLP_IN_PAD = 32;  // network input width (zero padded)
constexpr int MLP_HID = 64;
constexpr int MLP_OUT = 16;     // network output width (padded)
constexpr int MLP_NOUT = 3;     // outputs used
// packed FP32 parameters: W1 (32x64), b1, W2 (64x64), b2, W3 (64x16), b3, row-major
constexpr int MLP_W1 = 0;
constexpr int MLP_B1 = MLP_W1 + MLP_IN_PAD * MLP_HID;
constexpr int MLP_W2 = MLP_B1 + MLP_HID;
constexpr int MLP_B2 = MLP_W2 + MLP_HID * MLP_HID;
constexpr int MLP_W3 = MLP_B2 + MLP_HID;
constexpr int MLP_B3 = MLP_W3 + MLP_HID * MLP_OUT;
constexpr int MLP_NPARAM = MLP_B3 + MLP_OUT;
constexpr int MLP_MAX_BLOCKS = 256;
constexpr int MLP_WAVES = 4;           // waves per workgroup of the MLP kernels
// per-wave partial gradients (MLP_NPARAM floats each) and losses of one
// gradient evaluation: at most MLP_MAX_BLOCKS * MLP_WAVES waves
constexpr size_t MLP_PART_FLOATS = (size_t)MLP_MAX_BLOCKS * MLP_WAVES * MLP_NPARAM;
constexpr size_t MLP_LPART_FLOATS = (size_t)MLP_MAX_BLOCKS * MLP_WAVES;

struct MlpState {
  float* W = nullptr;           // FP32 masters
  float* m = nullptr;           // Adam first moments
  float* v = nullptr;           // Adam second moments
  float* grad = nullptr;        // last gradient
  float* part = nullptr;        // per-wave partial gradients
  float* lpart = nullptr;       // per-wave partial losses
  float* loss = nullptr;        // device scalar
  uint16_t* W1b = nullptr;      // bf16 copies used by the MFMA kernels
  uint16_t* W2b = nullptr;
  uint16_t* W3b = nullptr;
  float* mean = nullptr;        // feature normalisation
  float* istd = nullptr;
  int t = 0;                    // Adam step count
  bool set = false;
};

void mlp_refresh_bf16(const MlpState& s, hipStream_t st);
void mlp_forward(const MlpState& s, const float* X, int B, float* Y, hipStream_t st);
void mlp_gradient(const MlpState& s, const float* X, const float* T, const int* idx, int B, float* grad,
                  float* loss, hipStream_t st);
// The same with caller-provided partial buffers (part: MLP_PART_FLOATS,
// lpart: MLP_LPART_FLOATS floats); every partial read is written first.
void mlp_gradient_into(const MlpState& s, const float* X, const float* T, const int* idx, int B, float* grad,
                       float* loss, float* part, float* lpart, hipStream_t st);
void mlp_adam(MlpState& s, const float* grad, float lr, hipStream_t st);
void mlp_stats(MlpState& s, const float* X, int N, hipStream_t st);
// Features at the predictor xt; estore: the element store of an element-
// Hessian pass at xt in precision prec (0 float64, 1 float32) with scale s_el.
void launch_features(const MeshView& mv, const double* xt, const double* x0, double h, double E, int prec,
                     const void* estore, double s_el, double ell, const int* nptr, const int* nidx,
                     const double* Xr, float* out, const int* rowmap, hipStream_t st);
void launch_targets(const MeshView& mv, const double* xn, const double* xt, double ell, const int* rowmap,
                    float* T, hipStream_t st);
// The learned proposal: x~ + corr + ds * ell * Delta on free vertices (corr:
// the mesh's last step correction, MeshView::corr; ds = 0: the correction
// alone).
void launch_proposal(int n, int nf, const double* xt, const double* corr, const float* delta, double ell,
                     double ds, double* xp, hipStream_t st);
// x~ + corr in caller order (n x 3), the base the proposal adds ell * Delta to.
void launch_base_user(const MeshView& mv, const int* vperm, const double* xt, double* x_user, hipStream_t st);

}  // namespace cc
