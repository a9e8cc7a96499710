// Transfer matrix of the Trotter-Suzuki form in a parity sector (paper:
// Sec. 2.2, the EDQSG product; App. D, the parity-aware basis): kernels
// launched by the C ABI.  Vectors are float64 over the 2^(L^2-1) sector
// basis states, index n = the spins of sites 0 .. L^2-2 (bit j set: S_j = -1;
// the last site's spin is +1).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace qsg {

constexpr uint32_t kTmMaxL = 5;                       // 2^24 doubles per vector
constexpr uint32_t kTmMaxSites = kTmMaxL * kTmMaxL;
constexpr uint32_t kTmTable = 2 * kTmMaxSites + 1;    // unsatisfied bonds 0 .. 2 L^2

struct TmParams {
    uint32_t L, n;            // n = L^2 - 1 sector bits
    uint32_t not_last_col, last_col, not_last_row, last_row, all;  // site masks
    uint32_t jxm, jym;        // bit j: J = -1 on bond (j, +x) / (j, +y)
    double jp, jm;            // site factor jp 1 + jm sigma^X
    double jm_last;           // parity * jm: the last site's round
    double wtab[kTmTable];    // exp(k (L^2 - u)) = exp(k Bsp / 2), u unsatisfied bonds
};

// out = T in (in == out allowed).  Two launches for L = 4 and L = 5,
// one for L <= 3.
hipError_t launch_tm_apply(const TmParams& P, const double* in, double* out, hipStream_t s);

// out = the Walsh-Hadamard transform of in^2 elementwise over the n index
// bits: out[m] = sum_k in[k]^2 (-1)^popcount(k & m) (in == out allowed; the
// same passes as the product with the factor (a, b) -> (a + b, a - b)).
hipError_t launch_tm_wht_squares(const TmParams& P, const double* in, double* out, hipStream_t s);
// out[0..2] = sum_e w[3e + i] (W[mask[e]] / W[0])^2 for i = 0, 1, 2 (one
// block, fixed order).
hipError_t launch_tm_corr(const double* W, const uint32_t* mask, const double* w, uint32_t n,
                          double* out, hipStream_t s);

// Lanczos support, float64, deterministic (fixed reduction order).
constexpr uint32_t kTmDotBlocks = 512;  // partial sums per dot product
// h[i] = <V[i], w> for i < nv (V: nv vectors of N, contiguous); partial:
// nv * kTmDotBlocks doubles.
hipError_t launch_tm_dots(const double* V, uint32_t nv, size_t N, const double* w,
                          double* partial, double* h, hipStream_t s);
// w -= sum_i h[i] V[i]
hipError_t launch_tm_update(const double* V, uint32_t nv, size_t N, const double* h, double* w,
                            hipStream_t s);
// v = w / sqrt(*nrm2)
hipError_t launch_tm_scale(const double* w, size_t N, const double* nrm2, double* v, hipStream_t s);
// v = seeded uniform values in [-1, 1) (splitmix64 of seed and index)
hipError_t launch_tm_random(double* v, size_t N, uint64_t seed, hipStream_t s);
// out = sum_i y[i] V[i]
hipError_t launch_tm_combine(const double* V, uint32_t nv, size_t N, const double* y, double* out,
                             hipStream_t s);

// Host side: records the failure of a context-free entry point.
int32_t report_error(int32_t code, const char* fmt, ...);

}  // namespace qsg
