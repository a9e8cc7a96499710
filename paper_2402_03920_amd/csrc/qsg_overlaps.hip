// Euclidean-time overlaps of a slot's configuration (paper: App. E, the
// tau-dependent Q2, Q4 and F).  For a replica (lane) a and slices tau1,
// tau1 + tau: q_x = S_{x,tau1} S_{x,tau1+tau}, Qt = sum_x q_x, column sums
// C_x1 = sum_x2 q and row sums R_x2 = sum_x1 q.  One launch adds, for every
// requested tau, the integer contributions
//   q2[a][i] += sum_tau1 Qt^2,  q4[a][i] += sum_tau1 Qt^4,
//   A[i][d]  += sum_{a,tau1} sum_x1 C_x1 C_{x1+d},  B[i][d] likewise for R,
// from which Q2, Q4 and F(tau) follow (|sum_x e^{2 pi i x1/L} q_x|^2 =
// sum_d A-term(d) cos(2 pi d/L)).  All sums are integers, so the result does
// not depend on the order of the atomics.
//
// Layout: a wave handles one (tau1, tau) pair with lane j = replica j; the
// words of both slices are wave-uniform loads, bit j is the lane's spin.
// Column sums live in registers (L <= 32, unrolled), row sums in LDS.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "qsg_overlaps.h"

namespace qsg {
namespace {

constexpr int kOvWaves = 4;  // waves (tau1 values) per block

__global__ void __launch_bounds__(64 * kOvWaves)
k_tau_overlaps(const uint64_t* __restrict__ spins, uint32_t L, uint32_t Ltau, TauList taus,
               int64_t* __restrict__ out) {
    __shared__ int32_t rows[kOvWaves][kOvMaxL][64];
    __shared__ int32_t cols[kOvWaves][kOvMaxL][64];
    __shared__ int32_t redA[kOvWaves][kOvMaxL];
    __shared__ int32_t redB[kOvWaves][kOvMaxL];
    __shared__ int64_t red2[kOvWaves][64], red4[kOvWaves][64];
    // blockIdx.z: the slot, counted from the first one requested; each slot
    // has its own output block q2 [64][n], q4 [64][n], A [n][L], B [n][L]
    const uint32_t P = L * L;
    const uint64_t* __restrict__ S = spins + (size_t)blockIdx.z * P * Ltau;
    int64_t* __restrict__ q2 = out + (size_t)blockIdx.z * taus.n * (128 + 2 * L);
    int64_t* __restrict__ q4 = q2 + 64 * (size_t)taus.n;
    int64_t* __restrict__ A = q4 + 64 * (size_t)taus.n;
    int64_t* __restrict__ B = A + (size_t)taus.n * L;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t i = blockIdx.y;
    const uint32_t tau = taus.t[i];
    const uint32_t tau1 = blockIdx.x * kOvWaves + w;
    const bool live = tau1 < Ltau;  // wave-uniform
    int32_t C[kOvMaxL];
#pragma unroll
    for (int x = 0; x < kOvMaxL; ++x) C[x] = 0;
    int64_t Qt = 0;
    if (live) {
        uint32_t tau2 = tau1 + tau;
        if (tau2 >= Ltau) tau2 -= Ltau;
        const uint64_t* __restrict__ s1 = S + (size_t)tau1 * P;
        const uint64_t* __restrict__ s2 = S + (size_t)tau2 * P;
        for (uint32_t y = 0; y < L; ++y) {
            int32_t row = 0;
#pragma unroll
            for (int x = 0; x < kOvMaxL; ++x) {
                if ((uint32_t)x < L) {
                    const uint64_t d = s1[y * L + x] ^ s2[y * L + x];
                    const int32_t q = 1 - 2 * (int32_t)((d >> lane) & 1u);
                    row += q;
                    C[x] += q;
                }
            }
            rows[w][y][lane] = row;
            Qt += row;
        }
#pragma unroll
        for (int x = 0; x < kOvMaxL; ++x)
            if ((uint32_t)x < L) cols[w][x][lane] = C[x];
    }
    __syncthreads();
    // per lane: A(d) = sum_x1 C_x1 C_{x1+d}, B(d) = sum_x2 R_x2 R_{x2+d}; then
    // the wave's total over its 64 lanes
    for (uint32_t d = 0; d < L; ++d) {
        int32_t a = 0, b = 0;
        if (live) {
#pragma unroll
            for (int x = 0; x < kOvMaxL; ++x) {
                if ((uint32_t)x < L) {
                    uint32_t xd = (uint32_t)x + d;
                    if (xd >= L) xd -= L;
                    a += C[x] * cols[w][xd][lane];
                }
            }
            for (uint32_t y = 0; y < L; ++y) {
                uint32_t yd = y + d;
                if (yd >= L) yd -= L;
                b += rows[w][y][lane] * rows[w][yd][lane];
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            a += __shfl_xor(a, off, 64);
            b += __shfl_xor(b, off, 64);
        }
        if (lane == 0) {
            redA[w][d] = a;
            redB[w][d] = b;
        }
    }
    const int64_t Q2 = Qt * Qt;
    red2[w][lane] = Q2;
    red4[w][lane] = Q2 * Q2;
    __syncthreads();
    if (w == 0) {
        int64_t s2 = 0, s4 = 0;
#pragma unroll
        for (int k = 0; k < kOvWaves; ++k) {
            s2 += red2[k][lane];
            s4 += red4[k][lane];
        }
        atomicAdd((unsigned long long*)&q2[(size_t)lane * taus.n + i], (unsigned long long)s2);
        atomicAdd((unsigned long long*)&q4[(size_t)lane * taus.n + i], (unsigned long long)s4);
        if (lane < L) {
            int64_t sa = 0, sb = 0;
#pragma unroll
            for (int k = 0; k < kOvWaves; ++k) {
                sa += redA[k][lane];
                sb += redB[k][lane];
            }
            atomicAdd((unsigned long long*)&A[(size_t)i * L + lane], (unsigned long long)sa);
            atomicAdd((unsigned long long*)&B[(size_t)i * L + lane], (unsigned long long)sb);
        }
    }
}

}  // namespace

hipError_t launch_tau_overlaps(const uint64_t* slot_spins, uint32_t n_slots, uint32_t L,
                               uint32_t Ltau, const TauList& taus, int64_t* out, hipStream_t s) {
    if (taus.n == 0 || n_slots == 0) return hipSuccess;
    const dim3 grid((Ltau + kOvWaves - 1) / kOvWaves, taus.n, n_slots);
    hipLaunchKernelGGL(k_tau_overlaps, grid, dim3(64 * kOvWaves), 0, s, slot_spins, L, Ltau, taus,
                       out);
    return hipGetLastError();
}

}  // namespace qsg
