// Ladder-predicting MLP: forward, backward, loss, Adam and ladder decode.
//
// Network 6 -> 128 -> 128 -> 128 -> 32 with exact-erf GELU after the hidden
// layers.  Parameters are FP32 master values (flat layout W1[6][128], b1,
// W2[128][128], b2, W3[128][128], b3, W4[128][32], b4; W[k][n] maps input k
// to output n) with an optional BF16 copy.  With the BF16 copy, every GEMM
// operand is rounded to bfloat16 (nearest even) and products accumulate in
// FP32; bias, GELU, loss and Adam are FP32.  Without it the same kernels run
// in FP32 throughout.
//
// The matrices are at most [B x 128] x [128 x 128]: latency-bound, so each
// kernel is a plain one-thread-per-output loop with coalesced weight reads;
// everything is deterministic (no float atomics).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>

#include "qsg_mlp.h"

namespace qsg {
namespace {

__device__ __forceinline__ float bf16_round(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xFFFF0000u);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
    return __uint_as_float((uint32_t)h << 16);
}
__device__ __forceinline__ uint16_t f32_to_bf16(float x) {
    return (uint16_t)(__float_as_uint(bf16_round(x)) >> 16);
}
__device__ __forceinline__ float gelu(float x) {
    return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_grad(float x) {
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) +
           x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

struct Layer {
    int K, N;
    size_t w_off, b_off;
};

__host__ __device__ inline Layer layer(int l) {
    const int K[4] = {kMlpIn, kMlpHidden, kMlpHidden, kMlpHidden};
    const int N[4] = {kMlpHidden, kMlpHidden, kMlpHidden, kMlpOut};
    size_t off = 0;
    for (int i = 0; i < l; ++i) off += (size_t)K[i] * N[i] + N[i];
    return Layer{K[l], N[l], off, off + (size_t)K[l] * N[l]};
}

// out[b][n] = act(sum_k x[b][k] * W[k][n] + bias[n]); pre keeps the sum.
__global__ void k_linear_fwd(const float* __restrict__ X, int B, const float* __restrict__ Wf,
                             const uint16_t* __restrict__ Wh, const float* __restrict__ bias,
                             int K, int N, float* __restrict__ pre, float* __restrict__ out,
                             int act) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * N) return;
    const int b = i / N, n = i - b * N;
    const float* x = X + (size_t)b * K;
    float acc = 0.0f;
    if (Wh) {
        for (int k = 0; k < K; ++k) acc = fmaf(bf16_round(x[k]), bf16_to_f32(Wh[(size_t)k * N + n]), acc);
    } else {
        for (int k = 0; k < K; ++k) acc = fmaf(x[k], Wf[(size_t)k * N + n], acc);
    }
    acc += bias[n];
    if (pre) pre[i] = acc;
    out[i] = act ? gelu(acc) : acc;
}

// dpre = dy * gelu'(pre)
__global__ void k_gelu_bwd(const float* __restrict__ dy, const float* __restrict__ pre,
                           float* __restrict__ dpre, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dpre[i] = dy[i] * gelu_grad(pre[i]);
}

// dX[b][k] = sum_n dpre[b][n] * W[k][n]
__global__ void k_linear_bwd_data(const float* __restrict__ dpre, int B, const float* __restrict__ Wf,
                                  const uint16_t* __restrict__ Wh, int K, int N,
                                  float* __restrict__ dX) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * K) return;
    const int b = i / K, k = i - b * K;
    const float* d = dpre + (size_t)b * N;
    float acc = 0.0f;
    if (Wh) {
        for (int n = 0; n < N; ++n) acc = fmaf(bf16_round(d[n]), bf16_to_f32(Wh[(size_t)k * N + n]), acc);
    } else {
        for (int n = 0; n < N; ++n) acc = fmaf(d[n], Wf[(size_t)k * N + n], acc);
    }
    dX[i] = acc;
}

// dW[k][n] = sum_b x[b][k] * dpre[b][n]; db[n] = sum_b dpre[b][n]
__global__ void k_linear_bwd_weight(const float* __restrict__ X, const float* __restrict__ dpre,
                                    int B, int K, int N, int rounded, float* __restrict__ dW,
                                    float* __restrict__ db) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < K * N) {
        const int k = i / N, n = i - k * N;
        float acc = 0.0f;
        for (int b = 0; b < B; ++b) {
            const float x = X[(size_t)b * K + k];
            const float d = dpre[(size_t)b * N + n];
            acc = rounded ? fmaf(bf16_round(x), bf16_round(d), acc) : fmaf(x, d, acc);
        }
        dW[i] = acc;
    } else if (i < K * N + N) {
        const int n = i - K * N;
        float acc = 0.0f;
        for (int b = 0; b < B; ++b) acc += dpre[(size_t)b * N + n];
        db[n] = acc;
    }
}

// Per sample: KL(t || softmax(z[:31])) + (z[31] - logL)^2 and its gradient,
// scaled by 1/B (mean over the batch).
__global__ void k_loss(const float* __restrict__ z, const float* __restrict__ t,
                       const float* __restrict__ logL, int B, float* __restrict__ dz,
                       float* __restrict__ loss) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const float* zb = z + (size_t)b * kMlpOut;
    const float* tb = t + (size_t)b * kMlpInc;
    float m = zb[0];
    for (int l = 1; l < kMlpInc; ++l) m = fmaxf(m, zb[l]);
    float se = 0.0f, tsum = 0.0f;
    for (int l = 0; l < kMlpInc; ++l) {
        se += expf(zb[l] - m);
        tsum += tb[l];
    }
    const float lse = m + logf(se);
    float kl = 0.0f;
    const float inv_b = 1.0f / (float)B;
    for (int l = 0; l < kMlpInc; ++l) {
        const float s = expf(zb[l] - lse);
        if (tb[l] > 0.0f) kl += tb[l] * (logf(tb[l]) - (zb[l] - lse));
        dz[(size_t)b * kMlpOut + l] = (s * tsum - tb[l]) * inv_b;
    }
    const float d = zb[kMlpInc] - logL[b];
    dz[(size_t)b * kMlpOut + kMlpInc] = 2.0f * d * inv_b;
    loss[b] = kl + d * d;
}

__global__ void k_adam(float* __restrict__ p, uint16_t* __restrict__ ph, const float* __restrict__ g,
                       float* __restrict__ m, float* __restrict__ v, int n, float lr, float c1,
                       float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
    p[i] = pi;
    if (ph) ph[i] = f32_to_bf16(pi);
}

__global__ void k_to_bf16(const float* __restrict__ p, uint16_t* __restrict__ ph, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) ph[i] = f32_to_bf16(p[i]);
}

// Ladder from the 31 increment logits: log G_i = log Gmin + (log Gmax -
// log Gmin) * cumulative softmax; ends pinned exactly; predicted acceptance
// 1 - exp(z31)/31.
__global__ void k_decode(const float* __restrict__ z, const double* __restrict__ gmin,
                         const double* __restrict__ gmax, int B, double* __restrict__ ladder,
                         float* __restrict__ acc_pred) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const float* zb = z + (size_t)b * kMlpOut;
    double m = zb[0];
    for (int l = 1; l < kMlpInc; ++l) m = fmax(m, (double)zb[l]);
    double se = 0.0;
    for (int l = 0; l < kMlpInc; ++l) se += exp((double)zb[l] - m);
    const double lo = log(gmin[b]), hi = log(gmax[b]);
    double c = 0.0;
    double* out = ladder + (size_t)b * kMlpLadder;
    out[0] = gmin[b];
    for (int l = 0; l < kMlpInc - 1; ++l) {
        c += exp((double)zb[l] - m) / se;
        double gv = exp(lo + (hi - lo) * c);
        if (gv < out[l]) gv = out[l];
        out[l + 1] = gv;
    }
    out[kMlpLadder - 1] = gmax[b];
    if (out[kMlpLadder - 2] > gmax[b]) out[kMlpLadder - 2] = gmax[b];
    if (acc_pred) acc_pred[b] = 1.0f - expf(zb[kMlpInc]) / (float)kMlpInc;
}

inline unsigned blocks(long n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t mlp_forward(const float* pf, const uint16_t* ph, const float* x, int B, float* out,
                       float* ws, hipStream_t s) {
    const float* in = x;
    for (int l = 0; l < 4; ++l) {
        const Layer L = layer(l);
        float* pre = ws + mlp_ws_pre(l, B);
        float* act = (l < 3) ? ws + mlp_ws_act(l, B) : out;
        hipLaunchKernelGGL(k_linear_fwd, dim3(blocks((long)B * L.N, 128)), dim3(128), 0, s, in, B,
                           pf + L.w_off, ph ? ph + L.w_off : nullptr, pf + L.b_off, L.K, L.N, pre,
                           act, l < 3 ? 1 : 0);
        in = act;
    }
    return hipGetLastError();
}

hipError_t mlp_backward(const float* pf, const uint16_t* ph, const float* x, const float* ws,
                        const float* dout, int B, float* grads, float* scratch, hipStream_t s) {
    // scratch: gact [B][128] (gradient w.r.t. a hidden activation) and
    // gpre [B][128] (gradient w.r.t. a hidden pre-activation)
    float* gact = scratch;
    float* gpre_buf = scratch + (size_t)B * kMlpHidden;
    for (int l = 3; l >= 0; --l) {
        const Layer L = layer(l);
        const float* gpre = dout;  // output layer: no activation
        if (l < 3) {
            hipLaunchKernelGGL(k_gelu_bwd, dim3(blocks((long)B * L.N, 256)), dim3(256), 0, s, gact,
                               ws + mlp_ws_pre(l, B), gpre_buf, B * L.N);
            gpre = gpre_buf;
        }
        const float* xin = (l == 0) ? x : ws + mlp_ws_act(l - 1, B);
        hipLaunchKernelGGL(k_linear_bwd_weight, dim3(blocks((long)L.K * L.N + L.N, 128)), dim3(128),
                           0, s, xin, gpre, B, L.K, L.N, ph ? 1 : 0, grads + L.w_off,
                           grads + L.b_off);
        if (l > 0)
            hipLaunchKernelGGL(k_linear_bwd_data, dim3(blocks((long)B * L.K, 128)), dim3(128), 0, s,
                               gpre, B, pf + L.w_off, ph ? ph + L.w_off : nullptr, L.K, L.N, gact);
    }
    return hipGetLastError();
}

hipError_t mlp_loss(const float* z, const float* t, const float* logL, int B, float* dz,
                    float* loss, hipStream_t s) {
    hipLaunchKernelGGL(k_loss, dim3(blocks(B, 64)), dim3(64), 0, s, z, t, logL, B, dz, loss);
    return hipGetLastError();
}

hipError_t mlp_adam(float* p, uint16_t* ph, const float* g, float* m, float* v, uint32_t step,
                    float lr, hipStream_t s) {
    const float c1 = 1.0f - powf(0.9f, (float)step);
    const float c2 = 1.0f - powf(0.999f, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(blocks(kMlpParams, 256)), dim3(256), 0, s, p, ph, g, m, v,
                       kMlpParams, lr, c1, c2);
    return hipGetLastError();
}

hipError_t mlp_to_bf16(const float* p, uint16_t* ph, hipStream_t s) {
    hipLaunchKernelGGL(k_to_bf16, dim3(blocks(kMlpParams, 256)), dim3(256), 0, s, p, ph, kMlpParams);
    return hipGetLastError();
}

hipError_t mlp_decode(const float* z, const double* gmin, const double* gmax, int B, double* ladder,
                      float* acc_pred, hipStream_t s) {
    hipLaunchKernelGGL(k_decode, dim3(blocks(B, 64)), dim3(64), 0, s, z, gmin, gmax, B, ladder,
                       acc_pred);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Forward pass that allocates nothing: the activations live in a fixed
// device array of this library (one copy per GPU, held until the process
// ends) instead of a caller workspace.  In host code `scratch` names a
// host-side stand-in, not the device copy: its device address comes from
// hipGetSymbolAddress, looked up once per device with that device current,
// and only that address is ever passed to kernels.
// ---------------------------------------------------------------------------
__device__ __align__(256) float scratch[(size_t)kMlpNoAllocMaxBatch * (6 * kMlpHidden + kMlpOut)];
static_assert(sizeof(scratch) / sizeof(float) >= (size_t)6 * kMlpNoAllocMaxBatch * kMlpHidden +
                                                       (size_t)kMlpNoAllocMaxBatch * kMlpOut,
              "scratch must hold the forward workspace of the largest batch");

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t mlp_noalloc_scratch(float** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<float*>(p);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

hipError_t mlp_forward_noalloc(const float* pf, const uint16_t* ph, const float* x, int B,
                               float* out, hipStream_t s) {
    float* ws = nullptr;
    hipError_t e = mlp_noalloc_scratch(&ws);
    if (e != hipSuccess) return e;
    return mlp_forward(pf, ph, x, B, out, ws, s);
}

}  // namespace qsg
