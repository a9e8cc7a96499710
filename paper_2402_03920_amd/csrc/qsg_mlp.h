// Shapes and workspace layout of the ladder MLP (host and device).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace qsg {

constexpr int kMlpIn = 6;
constexpr int kMlpHidden = 128;
constexpr int kMlpOut = 32;
constexpr int kMlpInc = 31;     // increment logits; output 31 is the barrier head
constexpr int kMlpLadder = 32;  // ladder points
constexpr int kMlpParams = kMlpIn * kMlpHidden + kMlpHidden + 2 * (kMlpHidden * kMlpHidden + kMlpHidden) +
                           kMlpHidden * kMlpOut + kMlpOut;  // 38048

// Forward workspace (floats): per hidden layer l = 0..2 the pre-activation
// and the activation, each [B][128], then the output pre-activation [B][32].
__host__ __device__ inline size_t mlp_ws_pre(int l, int B) {
    return (size_t)(2 * l) * B * kMlpHidden;
}
__host__ __device__ inline size_t mlp_ws_act(int l, int B) {
    return (size_t)(2 * l + 1) * B * kMlpHidden;
}
__host__ __device__ inline size_t mlp_ws_floats(int B) {
    return (size_t)6 * B * kMlpHidden + (size_t)B * kMlpOut;
}

hipError_t mlp_forward(const float* pf, const uint16_t* ph, const float* x, int B, float* out,
                       float* ws, hipStream_t s);
// The same forward with its workspace in the library's fixed per-device
// array (batches of at most kMlpNoAllocMaxBatch; no allocation).
constexpr int kMlpNoAllocMaxBatch = 1024;
hipError_t mlp_forward_noalloc(const float* pf, const uint16_t* ph, const float* x, int B,
                               float* out, hipStream_t s);
hipError_t mlp_backward(const float* pf, const uint16_t* ph, const float* x, const float* ws,
                        const float* dout, int B, float* grads, float* scratch, hipStream_t s);
hipError_t mlp_loss(const float* z, const float* t, const float* logL, int B, float* dz,
                    float* loss, hipStream_t s);
hipError_t mlp_adam(float* p, uint16_t* ph, const float* g, float* m, float* v, uint32_t step,
                    float lr, hipStream_t s);
hipError_t mlp_to_bf16(const float* p, uint16_t* ph, hipStream_t s);
hipError_t mlp_decode(const float* z, const double* gmin, const double* gmax, int B, double* ladder,
                      float* acc_pred, hipStream_t s);

}  // namespace qsg
