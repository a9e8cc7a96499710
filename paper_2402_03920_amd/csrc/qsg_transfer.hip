// Transfer matrix in a parity sector (paper: Sec. 2.2, the EDQSG product;
// App. D, the parity-aware basis), float64:
//
//   out = W B W in,  W = diag exp(k Bsp(n) / 2),
//   B = prod_{j < L^2-1} (jp + jm X_j) (jp + parity jm C),
//
// X_j flips bit j of the index, C complements all L^2 - 1 bits.  The factors
// of B commute, so they are applied in whatever order suits the memory
// layout: the complement round pairs tile t with its mirror tile and is done
// in the first pass, next to the first W.
//
// Layout: a vector is 2^n doubles (n = L^2 - 1), index = sector state.  A
// pass loads a block of states into registers, does the rounds of a few
// index bits in registers, transposes through LDS, does the next bits, and
// stores: every pass reads and writes the vector once.  L = 5 takes two
// passes (bits 0-11 with W and the complement round on 4096-state tiles;
// bits 12-23 with W on 32768 states of 64-byte rows), L = 4 two (0-7,
// 8-14), L <= 3 one small block.
// W is not stored: each element's unsatisfied-bond count u comes from its
// index with shifts, masks and two popcounts, and indexes a table of
// exp(k (L^2 - u)) staged in LDS.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "qsg_transfer.h"

namespace qsg {
namespace {

constexpr int kTile = 4096;
constexpr int kTmThreads = 256;

// Unsatisfied bonds (site, +x) and (site, +y) of the slice state n: the
// spins of the +x (+y) neighbours are n rotated within rows (columns).
__device__ __forceinline__ uint32_t unsat(const TmParams& P, uint32_t n) {
    const uint32_t nx = ((n >> 1) & P.not_last_col) | ((n << (P.L - 1)) & P.last_col);
    const uint32_t ny = ((n >> P.L) & P.not_last_row) | ((n << (P.L * (P.L - 1))) & P.last_row);
    return (uint32_t)__popc((n ^ nx ^ P.jxm) & P.all) + (uint32_t)__popc((n ^ ny ^ P.jym) & P.all);
}

__device__ __forceinline__ void stage_table(const TmParams& P, double* wt) {
    for (uint32_t i = threadIdx.x; i < kTmTable; i += blockDim.x) wt[i] = P.wtab[i];
}

// The factors of the bits of a register index, pairs (r, r | 2^q): the
// site factor (a, b) -> (jp a + jm b, jp b + jm a), or with kHad the
// Walsh-Hadamard factor (a, b) -> (a + b, a - b).
template <int R, bool kHad = false>
__device__ __forceinline__ void rounds(double (&x)[R], double jp, double jm) {
#pragma unroll
    for (int q = 1; q < R; q <<= 1) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (r & q) continue;
            const double a = x[r], b = x[r | q];
            if (kHad) {
                x[r] = a + b;
                x[r | q] = a - b;
            } else {
                x[r] = jp * a + jm * b;
                x[r | q] = jp * b + jm * a;
            }
        }
    }
}

// Bits 4-7 (and, with k12, 8-11) of a 4096-element tile whose bits 0-3 are
// done: thread tt holds e = r + 16 tt in register r.  Transpose through LDS
// so that each thread holds the 16 values of bits 4-7 for one (bits 0-3,
// bits 8-11), four rounds; with k12 transpose again to bits 8-11, four more
// rounds.  Stores are coalesced (consecutive threads, consecutive states).
template <bool k12, bool kHad>
__device__ __forceinline__ void finish_low_tile(double* lds, double (&x)[16], size_t base,
                                                uint32_t tt, const TmParams& P, double* out) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const uint32_t e = (uint32_t)r + 16 * tt;
        lds[e + (e >> 4)] = x[r];
    }
    __syncthreads();
    const uint32_t lo = threadIdx.x & 15, cc = threadIdx.x >> 4;
    double y[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        const uint32_t e = lo + 16 * (uint32_t)s + 256 * cc;
        y[s] = lds[e + (e >> 4)];
    }
    rounds<16, kHad>(y, P.jp, P.jm);
    if (!k12) {
#pragma unroll
        for (int s = 0; s < 16; ++s) out[base + lo + 16 * (uint32_t)s + 256 * cc] = y[s];
        return;
    }
    __syncthreads();  // every value read before the tile is rewritten
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        const uint32_t e = lo + 16 * (uint32_t)s + 256 * cc;
        lds[e + (e >> 4)] = y[s];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const uint32_t e = threadIdx.x + 256 * (uint32_t)q;
        y[q] = lds[e + (e >> 4)];
    }
    rounds<16, kHad>(y, P.jp, P.jm);
#pragma unroll
    for (int q = 0; q < 16; ++q) out[base + threadIdx.x + 256 * (uint32_t)q] = y[q];
}

// First pass (n >= 15): block b takes tile b and its mirror (indices
// N-1-i), applies W, the last site's round between mirrored elements and
// the rounds of bits 0-7 (k12: 0-11) of both tiles.  With kHad it squares
// the input and applies the Walsh-Hadamard factors of the same bits only.
// in == out is allowed: every element is read before any is written, and
// blocks touch disjoint tiles.
template <bool k12, bool kHad>
__global__ void __launch_bounds__(kTmThreads)
k_tm_first(const TmParams P, const double* in, double* out) {
    __shared__ double lds[kTile + kTile / 16];
    __shared__ double wt[kTmTable];
    stage_table(P, wt);
    const size_t N = (size_t)1 << P.n;
    const size_t base_a = (size_t)blockIdx.x * kTile;
    const size_t base_b = N - kTile - base_a;
    const uint32_t t = threadIdx.x;
    // element r of this thread in tile A is e = r + 16 t; its mirror
    // 4095 - e is element 15 - r of thread 255 - t's slot in tile B, which
    // this thread loads
    const uint32_t ea = 16 * t;
    const uint32_t eb = 16 * (255 - t);
    double xa[16], xb[16];
#pragma unroll
    for (int r = 0; r < 16; r += 2) {
        const double2 va = *reinterpret_cast<const double2*>(in + base_a + ea + r);
        const double2 vb = *reinterpret_cast<const double2*>(in + base_b + eb + r);
        xa[r] = va.x;
        xa[r + 1] = va.y;
        xb[r] = vb.x;
        xb[r + 1] = vb.y;
    }
    __syncthreads();  // table staged
    if (kHad) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            xa[r] *= xa[r];
            xb[r] *= xb[r];
        }
    } else {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            xa[r] *= wt[unsat(P, (uint32_t)(base_a + ea) + (uint32_t)r)];
            xb[r] *= wt[unsat(P, (uint32_t)(base_b + eb) + (uint32_t)r)];
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const double a = xa[r], b = xb[15 - r];
            xa[r] = P.jp * a + P.jm_last * b;
            xb[15 - r] = P.jp * b + P.jm_last * a;
        }
    }
    rounds<16, kHad>(xa, P.jp, P.jm);
    rounds<16, kHad>(xb, P.jp, P.jm);
    finish_low_tile<k12, kHad>(lds, xa, base_a, t, P, out);
    __syncthreads();  // LDS reused for the mirror tile
    finish_low_tile<k12, kHad>(lds, xb, base_b, 255 - t, P, out);
}

// Second pass of L = 5 (n = 24): bits 12-23 of the 32768 states
// base + h 2^12 + c, h < 4096, c < 8 consecutive (64-byte rows), in place,
// then W.  1024 threads hold 32 states each: bits 0-4 of h in registers,
// then (transpose) bits 5-9, then (transpose) bits 10-11.  Each transpose
// goes through 128 KiB of LDS in two halves (split by h bit 11, then bit 9);
// the first uses rows h ^ ((h >> 5) & 3) so that neither side conflicts
// on banks.  The grid (512 blocks) is a multiple of 16.
constexpr int kHiThreads = 1024;
constexpr int kHiCols = 8;

__device__ __forceinline__ uint32_t hi_row_a(uint32_t h) {  // h < 4096, bit 11 = half
    const uint32_t hp = h & 2047u;
    return hp ^ ((hp >> 5) & 3u);
}
__device__ __forceinline__ uint32_t hi_row_b(uint32_t h) {  // bit 9 = half: removed
    return (h & 511u) | ((h >> 10) << 9);
}

template <bool kHad>
__global__ void __launch_bounds__(kHiThreads)
k_tm_hi12(const TmParams P, double* __restrict__ out) {
    __shared__ double lds[2048 * kHiCols];
    __shared__ double wt[kTmTable];
    stage_table(P, wt);
    const uint32_t t = threadIdx.x;
    const uint32_t c = t & 7u;
    // Column blocks 2m and 2m+1 share every 128-byte line.  Workgroups are
    // dealt to the eight XCDs in turn, so physical blocks p and p + 8 run on
    // the same XCD at about the same time: give them the two halves, and the
    // second half of each line comes from that XCD's L2.
    const uint32_t p = blockIdx.x;
    const uint32_t lb = 2 * (8 * (p >> 4) + (p & 7u)) + ((p >> 3) & 1u);
    const size_t base = (size_t)lb * kHiCols;
    double x[32];
    // layout 1: h = r + 32 hb
    const uint32_t hb = t >> 3;
#pragma unroll
    for (int r = 0; r < 32; ++r) x[r] = out[base + ((size_t)((uint32_t)r + 32 * hb) << 12) + c];
    rounds<32, kHad>(x, P.jp, P.jm);
    // layout 2: h = hl + 32 s + 1024 hh, hl = bits 0-4, hh = bits 10-11
    const uint32_t hl = (t >> 3) & 31u, hh = t >> 8;
    const uint32_t half = t >> 9;  // h bit 11 in layouts 1 and 2
#pragma unroll
    for (uint32_t k = 0; k < 2; ++k) {
        __syncthreads();
        if (half == k) {
#pragma unroll
            for (int r = 0; r < 32; ++r)
                lds[hi_row_a((uint32_t)r + 32 * hb) * kHiCols + c] = x[r];
        }
        __syncthreads();
        if (half == k) {
#pragma unroll
            for (int s = 0; s < 32; ++s)
                x[s] = lds[hi_row_a(hl + 32 * (uint32_t)s + 1024 * hh) * kHiCols + c];
        }
    }
    rounds<32, kHad>(x, P.jp, P.jm);
    // layout 3: h = hm + 128 g + 1024 q, register 4 g + q, hm = bits 0-6
    const uint32_t hm = t >> 3;
#pragma unroll
    for (uint32_t k = 0; k < 2; ++k) {
        __syncthreads();
#pragma unroll
        for (int s = 16 * k; s < 16 * (int)k + 16; ++s)
            lds[hi_row_b(hl + 32 * (uint32_t)s + 1024 * hh) * kHiCols + c] = x[s];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const uint32_t g = 4 * k + (uint32_t)(j >> 2), q = (uint32_t)(j & 3);
            x[16 * k + j] = lds[hi_row_b(hm + 128 * g + 1024 * q) * kHiCols + c];
        }
    }
#pragma unroll
    for (int q = 1; q < 4; q <<= 1) {  // bits 10-11: register bits 0-1
#pragma unroll
        for (int r = 0; r < 32; ++r) {
            if (r & q) continue;
            const double a = x[r], b = x[r | q];
            x[r] = kHad ? a + b : P.jp * a + P.jm * b;
            x[r | q] = kHad ? a - b : P.jp * b + P.jm * a;
        }
    }
#pragma unroll
    for (int j = 0; j < 32; ++j) {
        const uint32_t g = (uint32_t)(j >> 2), q = (uint32_t)(j & 3);
        const size_t i = base + ((size_t)(hm + 128 * g + 1024 * q) << 12) + c;
        out[i] = kHad ? x[j] : x[j] * wt[unsat(P, (uint32_t)i)];
    }
}

// A pass over bits b0 .. b0 + 3 + MB, in place.  The block's elements are
// base + h 2^b0 + c, h < 2^(4+MB), c < C consecutive (C = 4096 / 2^(4+MB));
// the block index fills the bits between log2 C and b0 and above the pass.
// The last pass also applies W.
template <int MB, bool kLast, bool kHad>
__global__ void __launch_bounds__(kTmThreads)
k_tm_pass(const TmParams P, uint32_t b0, double* __restrict__ out) {
    constexpr int M = 4 + MB;
    constexpr int C = kTile >> M;
    constexpr int LOGC = 12 - M;
    constexpr int HB = 1 << MB;   // registers per group in the second half
    constexpr int G = 16 / HB;    // groups per thread in the second half
    constexpr int CP = C + 1;     // padded LDS row
    __shared__ double lds[(1 << M) * CP];
    __shared__ double wt[kTmTable];
    if (kLast && !kHad) stage_table(P, wt);
    const uint32_t nlow = b0 - LOGC;
    const size_t B = blockIdx.x;
    const size_t base = ((B & ((1u << nlow) - 1)) << LOGC) | ((B >> nlow) << (b0 + M));
    const size_t stride = (size_t)1 << b0;
    const uint32_t t = threadIdx.x;
    const uint32_t c = t % C, hh = t / C;
    double x[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) x[r] = out[base + ((uint32_t)r + 16 * hh) * stride + c];
    rounds<16, kHad>(x, P.jp, P.jm);
#pragma unroll
    for (int r = 0; r < 16; ++r) lds[((uint32_t)r + 16 * hh) * CP + c] = x[r];
    __syncthreads();
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const uint32_t u = t + kTmThreads * (uint32_t)g;
        const uint32_t cc = u % C, lo = u / C;
        double y[HB];
#pragma unroll
        for (int s = 0; s < HB; ++s) y[s] = lds[(lo + 16 * (uint32_t)s) * CP + cc];
        rounds<HB, kHad>(y, P.jp, P.jm);
#pragma unroll
        for (int s = 0; s < HB; ++s) {
            const size_t i = base + (lo + 16 * (uint32_t)s) * stride + cc;
            double v = y[s];
            if (kLast && !kHad) v *= wt[unsat(P, (uint32_t)i)];
            out[i] = v;
        }
    }
}

// n <= 8: one block, one element per thread, every round through LDS in the
// paper's order (W, bits 0 .. n-1, the last site, W); with kHad the squared
// input and the Walsh-Hadamard factors of bits 0 .. n-1 only.
template <bool kHad>
__global__ void __launch_bounds__(kTmThreads)
k_tm_small(const TmParams P, const double* in, double* out) {
    __shared__ double v[kTmThreads];
    __shared__ double wt[kTmTable];
    stage_table(P, wt);
    __syncthreads();
    const uint32_t N = 1u << P.n, t = threadIdx.x;
    const bool live = t < N;
    double x = 0.0;
    if (live) x = kHad ? in[t] * in[t] : in[t] * wt[unsat(P, t)];
    for (uint32_t j = 0; j < P.n; ++j) {
        if (live) v[t] = x;
        __syncthreads();
        if (live) {
            const double o = v[t ^ (1u << j)];
            x = kHad ? ((t >> j) & 1u ? o - x : x + o) : P.jp * x + P.jm * o;
        }
        __syncthreads();
    }
    if (kHad) {
        if (live) out[t] = x;
        return;
    }
    if (live) v[t] = x;
    __syncthreads();
    if (live) out[t] = (P.jp * x + P.jm_last * v[N - 1 - t]) * wt[unsat(P, t)];
}

// ---------------------------------------------------------------------------
// Lanczos support: deterministic dot products (fixed partial-sum layout and
// reduction order), updates, scaling, seeded start vectors.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const uint32_t w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (uint32_t i = 0; i < (blockDim.x >> 6); ++i) s += red[i];
    return s;  // valid in thread 0
}

__global__ void __launch_bounds__(kTmThreads)
k_tm_dots(const double* __restrict__ V, size_t N, const double* __restrict__ w,
          double* __restrict__ partial) {
    __shared__ double red[kTmThreads / 64];
    const double* __restrict__ v = V + (size_t)blockIdx.y * N;
    double acc = 0.0;
    for (size_t i = (size_t)blockIdx.x * kTmThreads + threadIdx.x; i < N;
         i += (size_t)gridDim.x * kTmThreads)
        acc += v[i] * w[i];
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) partial[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = s;
}

__global__ void __launch_bounds__(kTmThreads)
k_tm_reduce(const double* __restrict__ partial, uint32_t G, double* __restrict__ h) {
    __shared__ double red[kTmThreads / 64];
    double acc = 0.0;
    for (uint32_t i = threadIdx.x; i < G; i += kTmThreads) acc += partial[(size_t)blockIdx.x * G + i];
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) h[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kTmThreads)
k_tm_update(const double* __restrict__ V, uint32_t nv, size_t N, const double* __restrict__ h,
            double* __restrict__ w) {
    for (size_t i = (size_t)blockIdx.x * kTmThreads + threadIdx.x; i < N;
         i += (size_t)gridDim.x * kTmThreads) {
        double acc = w[i];
        for (uint32_t j = 0; j < nv; ++j) acc -= h[j] * V[(size_t)j * N + i];
        w[i] = acc;
    }
}

__global__ void __launch_bounds__(kTmThreads)
k_tm_scale(const double* __restrict__ w, size_t N, const double* __restrict__ nrm2,
           double* __restrict__ v) {
    const double inv = 1.0 / sqrt(nrm2[0]);
    for (size_t i = (size_t)blockIdx.x * kTmThreads + threadIdx.x; i < N;
         i += (size_t)gridDim.x * kTmThreads)
        v[i] = w[i] * inv;
}

// splitmix64 (Steele, Lea and Flood, OOPSLA 2014) of seed + (i+1) * golden
// gamma: 53 bits to a double in [-1, 1).
__global__ void __launch_bounds__(kTmThreads)
k_tm_random(double* __restrict__ v, size_t N, uint64_t seed) {
    for (size_t i = (size_t)blockIdx.x * kTmThreads + threadIdx.x; i < N;
         i += (size_t)gridDim.x * kTmThreads) {
        uint64_t z = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        v[i] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
    }
}

__global__ void __launch_bounds__(kTmThreads)
k_tm_combine(const double* __restrict__ V, uint32_t nv, size_t N, const double* __restrict__ y,
             double* __restrict__ out) {
    for (size_t i = (size_t)blockIdx.x * kTmThreads + threadIdx.x; i < N;
         i += (size_t)gridDim.x * kTmThreads) {
        double acc = 0.0;
        for (uint32_t j = 0; j < nv; ++j) acc += y[j] * V[(size_t)j * N + i];
        out[i] = acc;
    }
}

uint32_t stream_blocks(size_t N) {
    const size_t b = (N + kTmThreads - 1) / kTmThreads;
    return (uint32_t)(b < 4096 ? b : 4096);
}

template <bool kHad>
hipError_t launch_passes(const TmParams& P, const double* in, double* out, hipStream_t s) {
    if (P.n <= 8) {
        hipLaunchKernelGGL(k_tm_small<kHad>, dim3(1), dim3(kTmThreads), 0, s, P, in, out);
        return hipGetLastError();
    }
    const size_t N = (size_t)1 << P.n;
    if (P.n == 15) {  // bits 0-7, then 8-14
        hipLaunchKernelGGL((k_tm_first<false, kHad>), dim3((uint32_t)(N / (2 * kTile))),
                           dim3(kTmThreads), 0, s, P, in, out);
        hipLaunchKernelGGL((k_tm_pass<3, true, kHad>), dim3((uint32_t)(N / kTile)), dim3(kTmThreads),
                           0, s, P, 8u, out);
    } else {          // n == 24: bits 0-11, then 12-23
        hipLaunchKernelGGL((k_tm_first<true, kHad>), dim3((uint32_t)(N / (2 * kTile))),
                           dim3(kTmThreads), 0, s, P, in, out);
        hipLaunchKernelGGL(k_tm_hi12<kHad>, dim3((uint32_t)(N / (4096 * kHiCols))), dim3(kHiThreads),
                           0, s, P, out);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_tm_apply(const TmParams& P, const double* in, double* out, hipStream_t s) {
    return launch_passes<false>(P, in, out, s);
}

hipError_t launch_tm_wht_squares(const TmParams& P, const double* in, double* out, hipStream_t s) {
    return launch_passes<true>(P, in, out, s);
}

namespace {

// Q2, Q4 and F sums from the transform: entry e adds wq2[e], wq4[e], wf[e]
// times (W[mask[e]] / W[0])^2; one block, fixed order.
__global__ void __launch_bounds__(kTmThreads)
k_tm_corr(const double* __restrict__ W, const uint32_t* __restrict__ mask,
          const double* __restrict__ wts, uint32_t n, double* __restrict__ out) {
    __shared__ double red[kTmThreads / 64];
    const double inv = 1.0 / W[0];
    double a2 = 0.0, a4 = 0.0, af = 0.0;
    for (uint32_t e = threadIdx.x; e < n; e += kTmThreads) {
        const double r = W[mask[e]] * inv;
        const double r2 = r * r;
        a2 += wts[3 * e] * r2;
        a4 += wts[3 * e + 1] * r2;
        af += wts[3 * e + 2] * r2;
    }
    const double s2 = block_sum(a2, red);
    __syncthreads();
    const double s4 = block_sum(a4, red);
    __syncthreads();
    const double sf = block_sum(af, red);
    if (threadIdx.x == 0) {
        out[0] = s2;
        out[1] = s4;
        out[2] = sf;
    }
}

}  // namespace

hipError_t launch_tm_corr(const double* W, const uint32_t* mask, const double* wts, uint32_t n,
                          double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_tm_corr, dim3(1), dim3(kTmThreads), 0, s, W, mask, wts, n, out);
    return hipGetLastError();
}

hipError_t launch_tm_dots(const double* V, uint32_t nv, size_t N, const double* w, double* partial,
                          double* h, hipStream_t s) {
    hipLaunchKernelGGL(k_tm_dots, dim3(kTmDotBlocks, nv), dim3(kTmThreads), 0, s, V, N, w, partial);
    hipLaunchKernelGGL(k_tm_reduce, dim3(nv), dim3(kTmThreads), 0, s, partial, kTmDotBlocks, h);
    return hipGetLastError();
}

hipError_t launch_tm_update(const double* V, uint32_t nv, size_t N, const double* h, double* w,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_tm_update, dim3(stream_blocks(N)), dim3(kTmThreads), 0, s, V, nv, N, h, w);
    return hipGetLastError();
}

hipError_t launch_tm_scale(const double* w, size_t N, const double* nrm2, double* v, hipStream_t s) {
    hipLaunchKernelGGL(k_tm_scale, dim3(stream_blocks(N)), dim3(kTmThreads), 0, s, w, N, nrm2, v);
    return hipGetLastError();
}

hipError_t launch_tm_random(double* v, size_t N, uint64_t seed, hipStream_t s) {
    hipLaunchKernelGGL(k_tm_random, dim3(stream_blocks(N)), dim3(kTmThreads), 0, s, v, N, seed);
    return hipGetLastError();
}

hipError_t launch_tm_combine(const double* V, uint32_t nv, size_t N, const double* y, double* out,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_tm_combine, dim3(stream_blocks(N)), dim3(kTmThreads), 0, s, V, nv, N, y,
                       out);
    return hipGetLastError();
}

}  // namespace qsg
