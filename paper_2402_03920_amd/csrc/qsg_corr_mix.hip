// Finite-L_tau estimates of the ground-state correlations (paper: App. E;
// EDQSG reports them for a list of Euclidean lengths): with the leading
// even and odd eigenpairs, a slice of a periodic prism of L_tau slices is
// the mixture (1 - w) |e><e| + w |o><o|, w = lambda_o^L_tau / (lambda_e^L_tau
// + lambda_o^L_tau), so every correlation mixes, R = (1 - w) R_e + w R_o,
// and Q2, Q4, F follow from the mixed correlations.  R_e and R_o are the
// Walsh-Hadamard transforms of the squared amplitudes (computed by the
// transfer-matrix passes), normalised by their value at 0.  One block per
// weight, fixed summation order.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "qsg_corr_mix.h"

namespace qsg {
namespace {

constexpr int kMixThreads = 256;

__global__ void __launch_bounds__(kMixThreads)
k_tm_corr_mixed(const double* __restrict__ We, const double* __restrict__ Wo,
                const uint32_t* __restrict__ mask, const double* __restrict__ wts, uint32_t n,
                const double* __restrict__ w_odd, double* __restrict__ out) {
    __shared__ double red[3][kMixThreads / 64];
    const double w = w_odd[blockIdx.x];
    const double ce = (1.0 - w) / We[0], co = w / Wo[0];
    double a2 = 0.0, a4 = 0.0, af = 0.0;
    for (uint32_t e = threadIdx.x; e < n; e += kMixThreads) {
        const uint32_t m = mask[e];
        const double r = ce * We[m] + co * Wo[m];
        const double r2 = r * r;
        a2 += wts[3 * e] * r2;
        a4 += wts[3 * e + 1] * r2;
        af += wts[3 * e + 2] * r2;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        a2 += __shfl_xor(a2, off, 64);
        a4 += __shfl_xor(a4, off, 64);
        af += __shfl_xor(af, off, 64);
    }
    const uint32_t wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][wv] = a2;
        red[1][wv] = a4;
        red[2][wv] = af;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double s = 0.0;
        for (int i = 0; i < kMixThreads / 64; ++i) s += red[threadIdx.x][i];
        out[3 * blockIdx.x + threadIdx.x] = s;
    }
}

}  // namespace

hipError_t launch_tm_corr_mixed(const double* We, const double* Wo, const uint32_t* mask,
                                const double* wts, uint32_t n, const double* w_odd,
                                uint32_t n_weights, double* out, hipStream_t s) {
    if (n_weights == 0) return hipSuccess;
    hipLaunchKernelGGL(k_tm_corr_mixed, dim3(n_weights), dim3(kMixThreads), 0, s, We, Wo, mask,
                       wts, n, w_odd, out);
    return hipGetLastError();
}

}  // namespace qsg
