// Learned warm start: per-constraint features, the MLP (BF16 MFMA
// inference, FP32 training kernels) and Adam.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "device_plan.hpp"

namespace ilves_ws {

constexpr int N_FEAT = 16;
constexpr int N_HID = 64;
// flat parameter layout: W1 [16][64], b1 [64], W2 [64][64], b2 [64], W3 [64], b3
constexpr int N_PARAMS = N_FEAT * N_HID + N_HID + N_HID * N_HID + N_HID + N_HID + 1;
// normalisation block: feature means [16], feature scales [16], output scale
constexpr int N_NORM = 2 * N_FEAT + 1;
constexpr int TRAIN_BS = 64;  // samples per training workgroup
constexpr int kChunk = 256;   // rows per chunk of the feature passes

// Features of every row of the listed row chunks ({molecule, first row},
// at most kChunk rows each; plan row order), and w_k = 1/m_a + 1/m_b.  Uses
// each molecule's workspace as scratch.
hipError_t launch_features(const ilves_dev::DevPlan& P, const int2* chunks, int32_t n_chunks, bool wide,
                           const double* r, const double* r_u, const double* mass, int32_t n_atoms,
                           unsigned char* ws, float* feat, float* w, hipStream_t stream);

// lambda_0 of every row: (t0 + scale * MLP((f - mean) / std)) / w, BF16
// MFMA with FP32 accumulation, written to lambda[cid[row]].
hipError_t launch_mlp_infer(const float* params, const float* norm, const float* feat, const float* w,
                            const int32_t* cid, int32_t n_rows, double* lambda, hipStream_t stream);

// FP32 reference-precision forward pass of normalised inputs x [n][16].
hipError_t launch_mlp_forward_f32(const float* params, const float* x, int32_t n, float* out, hipStream_t stream);

// Mean-squared-error gradient: L = 1/(2n) sum (out - y)^2.  work needs
// ceil(n / TRAIN_BS) * (N_PARAMS + 1) floats; grad receives N_PARAMS
// values, loss one.
hipError_t launch_mlp_grad_f32(const float* params, const float* x, const float* y, int32_t n, float* grad,
                               float* loss, float* work, hipStream_t stream);

// The same gradient with the partials in a file-scope device array of
// kStaticGradBlocks workgroup records (no caller workspace, no allocation):
// n <= kStaticGradBlocks * TRAIN_BS.  Calls that overlap on one GPU race.
constexpr int kStaticGradBlocks = 192;  // 12,288 samples, 4.1 MB per GPU
hipError_t launch_mlp_grad_f32_static(const float* params, const float* x, const float* y, int32_t n, float* grad,
                                      float* loss, hipStream_t stream);

// One Adam step on n parameters (step counts from 1).
hipError_t launch_mlp_adam(float* params, const float* grad, float* m, float* v, int32_t n, float lr, float beta1,
                           float beta2, float eps, int32_t step, hipStream_t stream);

}  // namespace ilves_ws
