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
// Layout: a wave handles (tau1, tau) pairs with lane j = replica j; the
// words of both slices are wave-uniform scalar loads, bit j is the lane's
// spin; one row of both slices per step of a loop over rows.  The kernel is
// instantiated per plane width L (even, <= 32), so the column sums live in
// registers with compile-time indices and the lagged products C_x C_{x+d}
// need no indexing at run time (the row sums pass through the lane's own
// LDS column once per plane); A(L-d) = A(d), so only lags 0 .. L/2 are
// formed.  A wave runs over several tau1 values
// (kOvPerWave) before its sums are reduced over lanes and waves and added
// to the output with one atomic per value and block.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "qsg_overlaps.h"

namespace qsg {
namespace {

constexpr int kOvWaves = 4;    // waves per block
constexpr int kOvPerWave = 8;  // tau1 values per wave
constexpr uint32_t kOvPerBlock = kOvWaves * kOvPerWave;

template <int L>
__global__ void __launch_bounds__(64 * kOvWaves)
k_tau_overlaps(const uint64_t* __restrict__ spins, uint32_t Ltau, TauList taus,
               int64_t* __restrict__ out) {
    constexpr int P = L * L;
    constexpr int H = L / 2;
    __shared__ int32_t redA[kOvWaves][H + 1];
    __shared__ int32_t redB[kOvWaves][H + 1];
    __shared__ int64_t red2[kOvWaves][64], red4[kOvWaves][64];
    __shared__ int32_t rows[kOvWaves][L][64];
    // blockIdx.z: the slot, counted from the first one requested; each slot
    // has its own output block q2 [64][n], q4 [64][n], A [n][L], B [n][L]
    const uint64_t* __restrict__ S = spins + (size_t)blockIdx.z * P * Ltau;
    int64_t* __restrict__ q2o = out + (size_t)blockIdx.z * taus.n * (128 + 2 * L);
    int64_t* __restrict__ q4o = q2o + 64 * (size_t)taus.n;
    int64_t* __restrict__ Ao = q4o + 64 * (size_t)taus.n;
    int64_t* __restrict__ Bo = Ao + (size_t)taus.n * L;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t i = blockIdx.y;
    const uint32_t tau = taus.t[i];
    const uint32_t t_end = min((blockIdx.x + 1) * kOvPerBlock, Ltau);
    int32_t Aacc[H + 1], Bacc[H + 1];
#pragma unroll
    for (int d = 0; d <= H; ++d) Aacc[d] = Bacc[d] = 0;
    int64_t s2 = 0, s4 = 0;
    for (uint32_t tau1 = blockIdx.x * kOvPerBlock + w; tau1 < t_end; tau1 += kOvWaves) {
        uint32_t tau2 = tau1 + tau;
        if (tau2 >= Ltau) tau2 -= Ltau;
        const uint64_t* __restrict__ s1 = S + (size_t)tau1 * P;
        const uint64_t* __restrict__ s2p = S + (size_t)tau2 * P;
        // counts of the sites with q = -1 per column (registers) and per
        // row (this lane's LDS column, read back once the plane is done)
        int32_t C[L], R[L];
#pragma unroll
        for (int x = 0; x < L; ++x) C[x] = 0;
#pragma unroll 1
        for (uint32_t y = 0; y < (uint32_t)L; ++y) {
            const uint64_t* __restrict__ a = s1 + y * L;
            const uint64_t* __restrict__ b = s2p + y * L;
            int32_t r = 0;
#pragma unroll
            for (int x = 0; x < L; ++x) {
                const int32_t bit = (int32_t)(((a[x] ^ b[x]) >> lane) & 1u);
                r += bit;
                C[x] += bit;
            }
            rows[w][y][lane] = r;
        }
#pragma unroll
        for (int y = 0; y < L; ++y) R[y] = rows[w][y][lane];
        int32_t tot = 0;
#pragma unroll
        for (int x = 0; x < L; ++x) {
            C[x] = L - 2 * C[x];
            R[x] = L - 2 * R[x];
            tot += R[x];
        }
        const int64_t Q2 = (int64_t)tot * tot;
        s2 += Q2;
        s4 += Q2 * Q2;
#pragma unroll
        for (int d = 0; d <= H; ++d) {
            int32_t a = 0, b = 0;
#pragma unroll
            for (int x = 0; x < L; ++x) {
                a += __mul24(C[x], C[(x + d) % L]);
                b += __mul24(R[x], R[(x + d) % L]);
            }
            Aacc[d] += a;
            Bacc[d] += b;
        }
    }
    // totals over the wave's lanes, then over the block's waves
#pragma unroll
    for (int d = 0; d <= H; ++d) {
        int32_t a = Aacc[d], b = Bacc[d];
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
    red2[w][lane] = s2;
    red4[w][lane] = s4;
    __syncthreads();
    if (w == 0) {
        int64_t t2 = 0, t4 = 0;
#pragma unroll
        for (int k = 0; k < kOvWaves; ++k) {
            t2 += red2[k][lane];
            t4 += red4[k][lane];
        }
        atomicAdd((unsigned long long*)&q2o[(size_t)lane * taus.n + i], (unsigned long long)t2);
        atomicAdd((unsigned long long*)&q4o[(size_t)lane * taus.n + i], (unsigned long long)t4);
        if (lane < (uint32_t)L) {
            const uint32_t d = lane <= (uint32_t)H ? lane : L - lane;  // A(L - d) = A(d)
            int64_t sa = 0, sb = 0;
#pragma unroll
            for (int k = 0; k < kOvWaves; ++k) {
                sa += redA[k][d];
                sb += redB[k][d];
            }
            atomicAdd((unsigned long long*)&Ao[(size_t)i * L + lane], (unsigned long long)sa);
            atomicAdd((unsigned long long*)&Bo[(size_t)i * L + lane], (unsigned long long)sb);
        }
    }
}

template <int L>
hipError_t launch_width(const uint64_t* slot_spins, uint32_t n_slots, uint32_t Ltau,
                        const TauList& taus, int64_t* out, hipStream_t s) {
    const dim3 grid((Ltau + kOvPerBlock - 1) / kOvPerBlock, taus.n, n_slots);
    hipLaunchKernelGGL(k_tau_overlaps<L>, grid, dim3(64 * kOvWaves), 0, s, slot_spins, Ltau, taus,
                       out);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_tau_overlaps(const uint64_t* slot_spins, uint32_t n_slots, uint32_t L,
                               uint32_t Ltau, const TauList& taus, int64_t* out, hipStream_t s) {
    if (taus.n == 0 || n_slots == 0) return hipSuccess;
    switch (L) {
#define QSG_OV_WIDTH(W) \
    case W: return launch_width<W>(slot_spins, n_slots, Ltau, taus, out, s);
        QSG_OV_WIDTH(2) QSG_OV_WIDTH(4) QSG_OV_WIDTH(6) QSG_OV_WIDTH(8) QSG_OV_WIDTH(10)
        QSG_OV_WIDTH(12) QSG_OV_WIDTH(14) QSG_OV_WIDTH(16) QSG_OV_WIDTH(18) QSG_OV_WIDTH(20)
        QSG_OV_WIDTH(22) QSG_OV_WIDTH(24) QSG_OV_WIDTH(26) QSG_OV_WIDTH(28) QSG_OV_WIDTH(30)
        QSG_OV_WIDTH(32)
#undef QSG_OV_WIDTH
        default: return hipErrorInvalidValue;
    }
}

}  // namespace qsg
