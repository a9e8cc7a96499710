// Internal layout shared by the host API and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace qsg {

// Per-(walker, lane) round-trip tracker; same layout as qsg_roundtrip.
struct RoundTrip {
    uint32_t state;
    uint32_t t_last;
    uint32_t count;
    uint32_t pad;
    uint64_t sum;
};

// Counters the energy pass accumulates per slot: unsatisfied space bonds and
// time bonds per lane, differing lane pairs per pair.
constexpr int kCntStride = 64 + 64 + 32;  // int32 per slot
// Per-slot measurement sums: Bsp[64], Bt[64], q[32], q^2[32] as int64.
constexpr int kSumStride = 192;
// Per-slot table: [0, 15) thresholds of the fifteen classes, [15] the class
// regime, [16, 24) the level picks (one byte per comparison level, most
// significant first, four to a word): for the seven classes of regimes 0-2,
// bits 0-6 mark the classes whose threshold has a 1 at that level, or, when
// more than three do, bits 0-6 mark those with a 0 and bit 7 is set.
constexpr int kThrStride = 32;
constexpr int kLevelPicks = 16;
// Histogram of the unsatisfied time bonds u = (V - Bt)/2 per slot, taken at
// every PT step before the exchanges: bin = u * kHistBins / (V + 1).
constexpr int kHistBins = 1024;

// Exact division by a fixed d for x < 2^31: q = mulhi(x, m) >> s, or
// x >> s when m == 0 (d a power of two).
struct Divisor {
    uint32_t m, s;
};

inline Divisor make_divisor(uint32_t d) {
    Divisor r{0, 0};
    uint32_t a = 0;
    while ((1ull << (a + 1)) <= d) ++a;  // a = floor(log2 d)
    if ((1u << a) == d) {
        r.s = a;
    } else {
        // d in (2^a, 2^(a+1)): m = ceil(2^(32+a)/d) < 2^32, exact for x < 2^31
        r.m = (uint32_t)(((1ull << (32 + a)) + d - 1) / d);
        r.s = a;
    }
    return r;
}

// Everything a kernel needs to know about one group.  Lives on the host
// (plain launches pass it by value) and in a device array (batched
// launches index it).
struct GroupDev {
    uint32_t L, Ltau, N, gid;
    uint32_t key0, key1;  // Monte Carlo key (mc_seed lo, hi)
    uint32_t V;           // words per slot = L*L*Ltau
    uint32_t sw_cap;      // entries per exchange table
    uint32_t log_cap;     // rows of the swap log
    uint32_t q_split;     // colour-pass schedule: Philox blocks before packing
    uint32_t tile;        // colour-pass schedule: tau planes per column walk (even, divides Ltau)
    uint32_t exch_all;    // PT energy: 0 time bonds (Gamma ladder), 1 all bonds (k ladder)
    uint32_t anti;        // 1: antiperiodic along tau (the wrapping time bond flips sign)
    uint32_t etile;       // energy pass, batched: tau planes per column walk (divides Ltau)
    Divisor div_half_plane, div_half_row, div_plane, div_row;
    Divisor div_blocks;   // colour-pass blocks per slot (sweep_blocks_per_slot(V, tile))
    uint64_t* spins;          // [N][Ltau][L][L]
    uint64_t* Jx;             // [L*L]
    uint64_t* Jy;             // [L*L]
    const uint64_t* jseed;    // [64] coupling keys
    uint32_t* thr;            // [N][kThrStride] thresholds, regime, level picks
    uint32_t* sw_thr;         // [N-1][sw_cap]
    uint32_t* sw_len;         // [N-1]
    uint32_t* sw_eq;          // [N-1]
    int32_t* cnt;             // [N][kCntStride]
    int32_t* E;               // [N][64][2] current (Bsp, Bt)
    uint32_t* walker;         // [N][64]
    RoundTrip* rt;            // [N walkers][64 lanes]
    uint64_t* acc;            // [N-1]
    uint64_t* swaplog;        // [log_cap][N-1]
    int64_t* sums;            // [N][kSumStride]
    uint64_t* lastmask;       // [N] masks of the latest PT step (+ any flag at [N-1])
    int32_t* meas;            // [N][kCntStride] scratch for on-demand measurement
    uint32_t* hist;           // [N][kHistBins]
};

// Launchers (qsg_kernels.hip).  All enqueue on `s` and return the launch
// status.  `ctr` is the device pair (sweeps done, PT steps done); sweep and
// PT kernels use ctr[0] + t_add and ctr[1] + p_add as their indices.
hipError_t launch_init_couplings(const GroupDev& g, hipStream_t s);
hipError_t launch_init_spins(const GroupDev& g, hipStream_t s);
hipError_t launch_init_state(const GroupDev& g, hipStream_t s);
// The colour pass follows the group's schedule G.q_split: Philox blocks every
// word goes through before the words still undecided are packed into the
// first waves of the block (16: no packing).  Results do not depend on it.
hipError_t launch_half_sweep(const GroupDev& g, uint32_t colour, const uint32_t* ctr,
                             uint32_t t_add, hipStream_t s);
hipError_t launch_energy(const GroupDev& g, int32_t* cnt, hipStream_t s);
hipError_t launch_pt(const GroupDev& g, const uint32_t* ctr, uint32_t p_add, hipStream_t s);
hipError_t launch_advance(uint32_t* ctr, uint32_t dt, uint32_t dp, hipStream_t s);
hipError_t launch_swap_apply(const GroupDev& g, hipStream_t s);
hipError_t launch_zero32(void* p, size_t n_words32, hipStream_t s);

hipError_t launch_philox(const uint32_t* in, uint32_t* out, uint32_t n, hipStream_t s);
hipError_t launch_philox_probe(uint32_t* out, uint32_t n, uint32_t blocks, uint64_t key,
                              hipStream_t s);

// Batched: one launch per pass over all groups.  `prefix[i]` is the first
// block of group i (prefix[n_groups] = total blocks).
// Group of a block and the block's index within the group.
struct BlockEntry {
    uint32_t gi, local;
};

struct BatchPlan {
    const GroupDev* groups;  // device array [n_groups]
    const uint32_t* prefix;  // device array [n_groups + 1]
    // optional device array [n_blocks]: every block's group and index in
    // it, so that a block of an ensemble of unequal groups finds its group
    // with one load instead of a search of `prefix`
    const BlockEntry* block_map;
    uint32_t n_groups;
    uint32_t n_blocks;
    // per_group > 0 when every group has exactly per_group blocks: a block
    // then finds its group by one scalar division (span divides by
    // per_group) instead of a search of `prefix`
    uint32_t per_group;
    Divisor span;
    // same_shape != 0 when every group's record equals `first` up to its
    // Philox identity (gid, key0, key1) and pointers that advance by
    // `stride` bytes from one group to the next: a block then builds its
    // record from this kernel argument instead of loading it first
    uint32_t same_shape;
    uint64_t stride;
    GroupDev first;
};

// Record i with its pointers moved back by `shift` bytes and its Philox
// identity cleared: equal for all groups of one shape (shift = i * stride).
inline bool same_but_identity(const GroupDev& a, const GroupDev& b, uint64_t shift) {
    auto ptr = [shift](const void* p, const void* q) {
        return (uint64_t)(uintptr_t)p == (uint64_t)(uintptr_t)q + shift;
    };
    auto div = [](Divisor x, Divisor y) { return x.m == y.m && x.s == y.s; };
    return a.L == b.L && a.Ltau == b.Ltau && a.N == b.N && a.V == b.V && a.sw_cap == b.sw_cap &&
           a.log_cap == b.log_cap && a.q_split == b.q_split && a.tile == b.tile &&
           a.exch_all == b.exch_all && a.etile == b.etile &&
           a.anti == b.anti && div(a.div_half_plane, b.div_half_plane) &&
           div(a.div_half_row, b.div_half_row) && div(a.div_plane, b.div_plane) &&
           div(a.div_row, b.div_row) && div(a.div_blocks, b.div_blocks) &&
           ptr(a.spins, b.spins) && ptr(a.Jx, b.Jx) && ptr(a.Jy, b.Jy) && ptr(a.jseed, b.jseed) &&
           ptr(a.thr, b.thr) && ptr(a.sw_thr, b.sw_thr) && ptr(a.sw_len, b.sw_len) &&
           ptr(a.sw_eq, b.sw_eq) && ptr(a.cnt, b.cnt) && ptr(a.E, b.E) &&
           ptr(a.walker, b.walker) && ptr(a.rt, b.rt) && ptr(a.acc, b.acc) &&
           ptr(a.swaplog, b.swaplog) && ptr(a.sums, b.sums) && ptr(a.lastmask, b.lastmask) &&
           ptr(a.meas, b.meas) && ptr(a.hist, b.hist);
}

// Set the plan's shared-shape fields from the host copy of the records
// (again whenever a record changes).
inline void set_plan_shape(BatchPlan& p, const GroupDev* records, uint32_t n_groups) {
    p.same_shape = 0;
    p.stride = 0;
    p.first = GroupDev{};
    if (n_groups == 0) return;
    const uint64_t base = (uint64_t)(uintptr_t)records[0].spins;
    const uint64_t stride = n_groups > 1 ? (uint64_t)(uintptr_t)records[1].spins - base : 0;
    for (uint32_t i = 0; i < n_groups; ++i)
        if (!same_but_identity(records[i], records[0], (uint64_t)i * stride)) return;
    p.same_shape = 1;
    p.stride = stride;
    p.first = records[0];
}

// The plan of a batched launch from the host copy of its prefix sums and
// of the group records.
inline BatchPlan make_plan(const GroupDev* groups, const uint32_t* d_prefix,
                           const uint32_t* prefix, uint32_t n_groups, const GroupDev* records) {
    BatchPlan p{};
    p.groups = groups;
    p.prefix = d_prefix;
    p.n_groups = n_groups;
    p.n_blocks = prefix[n_groups];
    const uint32_t first = n_groups ? prefix[1] - prefix[0] : 0;
    bool equal = first > 0;
    for (uint32_t i = 1; equal && i < n_groups; ++i) equal = prefix[i + 1] - prefix[i] == first;
    if (equal) {
        p.per_group = first;
        p.span = make_divisor(first);
    }
    set_plan_shape(p, records, n_groups);
    return p;
}
hipError_t launch_half_sweep_batched(const BatchPlan& plan, uint32_t colour, const uint32_t* ctr,
                                     uint32_t t_add, hipStream_t s);
hipError_t launch_energy_batched(const BatchPlan& plan, hipStream_t s);
// Fused sweeps over every slot (one block per slot, `slots.prefix` counts
// slots per group): n_sweeps sweeps in one launch; slots of at most
// lds_words words run from LDS.
hipError_t launch_chunk_fused(const BatchPlan& slots, const uint32_t* ctr, uint32_t n_sweeps,
                              uint32_t lds_words, hipStream_t s);
constexpr uint32_t kFusedLdsMaxWords = 7168;  // 56 KiB of spins per block
// Column-walk depth of the colour pass: the default and the largest allowed
// (tau planes per thread; each thread updates tile/2 words).
constexpr uint32_t kDefaultTile = 8;
constexpr uint32_t kMaxTile = 32;
// Largest power of two <= cap that divides Ltau (Ltau is even: at least 2).
inline uint32_t tile_for(uint32_t Ltau, uint32_t cap) {
    uint32_t t = 2;
    while (t * 2 <= cap && Ltau % (t * 2) == 0) t *= 2;
    return t;
}
hipError_t launch_pt_batched(const GroupDev* groups, uint32_t n_groups, const uint32_t* ctr,
                             uint32_t p_add, hipStream_t s);
hipError_t launch_swap_apply_batched(const BatchPlan& plan, hipStream_t s);

// Blocks one group needs in each pass (host and device agree on these).
// The colour pass gives each thread one column (x, y) of one tau tile of
// `tile` planes: V / tile threads per slot.
__host__ __device__ inline uint32_t sweep_blocks_per_slot(uint32_t V, uint32_t tile);
__host__ __device__ inline uint32_t energy_blocks_per_slot(uint32_t V, uint32_t words);
__host__ __device__ inline uint32_t swap_blocks(uint32_t V);

constexpr uint32_t kMaxSlots = 64;  // slots per group (the C ABI's QSG_MAX_GAMMA)
constexpr int kSweepBlock = 256;   // threads per block of a colour pass
constexpr uint32_t kWaveSize = 64;
// Energy pass: each thread walks one column through a tau tile of at most
// this many planes (batched launches; a launch for one group takes at most
// kEnergyPlanesSlot so that it still has enough blocks).
constexpr int kEnergyWords = 64;
constexpr int kEnergyPlanesSlot = 16;
constexpr int kEnergyBlock = 256;
constexpr int kSwapBlock = 256;

}  // namespace qsg

namespace qsg {
__host__ __device__ inline uint32_t sweep_blocks_per_slot(uint32_t V, uint32_t tile) {
    return (V / tile + kSweepBlock - 1) / kSweepBlock;
}
// The fused chunk kernel walks a slot's colour-c words block by block.
__host__ __device__ inline uint32_t fused_words_per_colour(uint32_t V) { return V / 2; }
// `planes` divides Ltau, so V / planes threads cover the slot exactly.
__host__ __device__ inline uint32_t energy_blocks_per_slot(uint32_t V, uint32_t planes) {
    return (V / planes + kEnergyBlock - 1) / kEnergyBlock;
}
__host__ __device__ inline uint32_t swap_blocks(uint32_t V) {
    return (V + kSwapBlock - 1) / kSwapBlock;
}
}  // namespace qsg
