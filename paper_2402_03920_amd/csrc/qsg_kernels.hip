// HIP kernels (gfx950, wave64) of the MCQSG Metropolis + parallel-tempering
// hot path.  Paper: Sec. 2.1 (multi-spin coding, checkerboard Metropolis,
// precomputed acceptance factors, parallel tempering), Sec. 2.1.1 (counter-
// based Philox4x32-10 random numbers tied to the lattice update).
//
// Multi-spin coding here packs 64 independent chains of one site into a
// uint64 (bit j = lane j), so a thread updates 64 spins with bitwise logic:
//   * unsatisfied bonds: u = s ^ neighbour ^ J (bit set <=> J S S' < 0);
//   * per-lane counts n_s (4 space bonds) and n_t (2 time bonds) as
//     bit-sliced adders, turned into 15 one-hot class masks;
//   * acceptance r_j <= thr[class_j]: lane numbers are bit-sliced over 32
//     levels (bit 31-b of r_j is bit j of level b), so all 64 comparisons run
//     together, most significant level first, and stop as soon as every lane
//     of the wave is decided.  One Philox block yields two levels.
// Nothing here is a dense contraction, so there is no matrix-core work: the
// pass is integer VALU work on data streamed from HBM.
#include <hip/hip_runtime.h>

#include "qsg_internal.h"

namespace qsg {
namespace {

constexpr uint32_t kM0 = 0xD2511F53u;
constexpr uint32_t kM1 = 0xCD9E8D57u;
constexpr uint32_t kW0 = 0x9E3779B9u;
constexpr uint32_t kW1 = 0xBB67AE85u;

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 products
// and xors with the key, the key advanced by the Weyl constants.  Each
// product is one v_mad_u64_u32 (both halves at once) and each three-way xor
// one v_bitop3_b32.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// In the colour pass only counter word 0 (the site) differs between lanes,
// so the first two rounds group their xors to keep the block-uniform parts
// on the scalar unit: round 0 has c.y, c.z, c.w uniform, round 1 c.x, c.y.
__device__ __forceinline__ uint4 philox(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)c.x * kM0;
        const uint64_t p1 = (uint64_t)c.z * kM1;
        const uint32_t h0 = (uint32_t)(p0 >> 32), h1 = (uint32_t)(p1 >> 32);
        if (r == 0)
            c = make_uint4(h1 ^ (c.y ^ k0), (uint32_t)p1, h0 ^ (c.w ^ k1), (uint32_t)p0);
        else if (r == 1)
            c = make_uint4(h1 ^ (c.y ^ k0), (uint32_t)p1, (h0 ^ k1) ^ c.w, (uint32_t)p0);
        else
            c = make_uint4(xor3(h1, c.y, k0), (uint32_t)p1, xor3(h0, c.w, k1), (uint32_t)p0);
        k0 += kW0;
        k1 += kW1;
    }
    return c;
}

__device__ __forceinline__ uint64_t lo_hi(uint32_t lo, uint32_t hi) {
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

// A group record read from memory by a batched kernel: every block reads one
// record, so its fields are block-uniform; moving them to scalar registers
// keeps all addressing and threshold logic on the scalar unit.
__device__ __forceinline__ GroupDev uniform_record(const GroupDev* __restrict__ p) {
    static_assert(sizeof(GroupDev) % 4 == 0, "record must be whole dwords");
    union {
        GroupDev g;
        uint32_t w[sizeof(GroupDev) / 4];
    } u;
    u.g = *p;
#pragma unroll
    for (int i = 0; i < (int)(sizeof(GroupDev) / 4); ++i) u.w[i] = __builtin_amdgcn_readfirstlane(u.w[i]);
    return u.g;
}

// Division of x < 2^31 by a block-uniform d >= 1 with a precomputed
// multiplier: q = mulhi(x, m) >> s (see make_divisor on the host).
__device__ __forceinline__ uint32_t fast_div(uint32_t x, Divisor d) {
    return d.m ? (__umulhi(x, d.m) >> d.s) : (x >> d.s);
}

// Classes (n_s, n_t) whose flip can raise the energy (dE > 0), for the three
// orderings of the two couplings; every other class has dE <= 0 and is
// always accepted.  Regime 0: kp > 2k, 1: k < kp <= 2k, 2: kp <= k.
template <int R> struct Classes;
template <> struct Classes<0> {
    static constexpr int n = 7;
    static constexpr int ns[7] = {0, 1, 2, 3, 4, 0, 1};
    static constexpr int nt[7] = {0, 0, 0, 0, 0, 1, 1};
};
template <> struct Classes<1> {
    static constexpr int n = 7;
    static constexpr int ns[7] = {0, 1, 2, 3, 0, 1, 0};
    static constexpr int nt[7] = {0, 0, 0, 0, 1, 1, 2};
};
template <> struct Classes<2> {
    static constexpr int n = 7;
    static constexpr int ns[7] = {0, 1, 2, 0, 1, 0, 1};
    static constexpr int nt[7] = {0, 0, 0, 1, 1, 2, 2};
};
template <> struct Classes<3> {  // any table: all fifteen classes
    static constexpr int n = 15;
    static constexpr int ns[15] = {0, 0, 0, 1, 1, 1, 2, 2, 2, 3, 3, 3, 4, 4, 4};
    static constexpr int nt[15] = {0, 1, 2, 0, 1, 2, 0, 1, 2, 0, 1, 2, 0, 1, 2};
};

__device__ __forceinline__ uint64_t all_if(uint32_t v, uint32_t bit) {
    return 0ull - (uint64_t)((v >> bit) & 1u);  // block-uniform 0 or ~0
}

// Three-input bitwise operation of gfx950 (v_bitop3_b32); the immediate is
// the truth table f(0xF0, 0xCC, 0xAA) of the operand order (a, b, c).
#define BITOP3(a, b, c, table) __builtin_amdgcn_bitop3_b32((a), (b), (c), (table))
constexpr int kAndOr = 0xEA;      // (a & b) | c
constexpr int kAndAndNot = 0x40;  // a & b & ~c
constexpr int kAndXnor = 0x90;    // a & ~(b ^ c)
constexpr int kXor3 = 0x96;       // a ^ b ^ c
constexpr int kMajority = 0xE8;   // at least two of a, b, c
constexpr int kXorAnd = 0x78;     // a ^ (b & c)
constexpr int kSelect = 0xCA;     // a ? b : c (bitwise)
constexpr int kAnd3 = 0x80;       // a & b & c
constexpr int kAndNotAnd = 0x20;  // a & ~b & c
constexpr int kNor3 = 0x01;       // ~(a | b | c)
constexpr int kEqEq = 0x81;       // a == b and a == c
constexpr int kNeNe = 0x18;       // a != b and a != c

template <int T>
__device__ __forceinline__ uint64_t bop3(uint64_t a, uint64_t b, uint64_t c) {
    return lo_hi(BITOP3((uint32_t)a, (uint32_t)b, (uint32_t)c, T),
                 BITOP3((uint32_t)(a >> 32), (uint32_t)(b >> 32), (uint32_t)(c >> 32), T));
}

// Per-word state of the comparison: the class planes it needs (bit-sliced
// n_s = s2 s1 s0 and one-hot planes of n_t = 0, 1, 2), the lanes accepted so
// far and the lanes still undecided.
struct WordState {
    uint32_t s;  // flat site index (RNG counter word 0)
    uint64_t w;  // centre word before the update
    uint64_t s0, s1, s2, nt0, nt1, nt2;
    uint64_t acc, und;
};

// LDS of a colour-pass block.  At the start of a call every thread writes
// its word's site, centre word and class planes to its own slot (the n_t = 1
// plane is not stored: the three n_t planes are one-hot), so they need not
// stay in registers through the comparison.  Words still undecided after
// the first levels are queued as (owner thread, accepted, undecided lanes)
// and finished by as few waves as possible, reading the rest from the
// owner's slot.  Two pairs of counters alternate between consecutive calls
// of a block: a slow thread may still be reading the previous call's count
// after a fast one has cleared the counters for the next call.
struct SweepQueue {
    uint32_t count[4];
    // per-thread slots
    uint32_t s[kSweepBlock];
    uint64_t w[kSweepBlock], s0[kSweepBlock], s1[kSweepBlock], s2[kSweepBlock];
    uint64_t nt0[kSweepBlock], nt2[kSweepBlock];
    // queue entries
    uint32_t owner[kSweepBlock];
    uint64_t acc[kSweepBlock], und[kSweepBlock];
};


// Spin and coupling words are addressed as base + 32-bit byte offset, so
// global accesses keep the base in SGPRs and only the offset in a VGPR.  The
// host rejects slots of more than 2^29 words, so a word index i < 2^29 gives
// a byte offset i * 8 < 2^32.  The fused kernel may hold a slot in LDS and
// addresses it generically.
typedef char __attribute__((address_space(1))) GlobalByte;
template <bool kGlobal>
__device__ __forceinline__ uint64_t load64(const uint64_t* base, uint32_t i) {
    if (kGlobal)
        return *(const uint64_t __attribute__((address_space(1)))*)((const GlobalByte*)base + i * 8u);
    return base[i];
}
template <bool kGlobal>
__device__ __forceinline__ void store64(uint64_t* base, uint32_t i, uint64_t v) {
    if (kGlobal)
        *(uint64_t __attribute__((address_space(1)))*)((GlobalByte*)base + i * 8u) = v;
    else
        base[i] = v;
}

// Site (x, y, tau): its six neighbours and four couplings, the unsatisfied
// bonds and their bit-sliced counts.
template <bool kGlobal>
__device__ __forceinline__ WordState load_site(const GroupDev& G, const uint64_t* __restrict__ S,
                                               uint32_t x, uint32_t y, uint32_t tau) {
    const uint32_t L = G.L;
    const uint32_t P = L * L;
    const uint32_t xp = (x + 1 == L) ? 0 : x + 1;
    const uint32_t xm = (x == 0) ? L - 1 : x - 1;
    const uint32_t yp = (y + 1 == L) ? 0 : y + 1;
    const uint32_t ym = (y == 0) ? L - 1 : y - 1;
    const uint32_t tp = (tau + 1 == G.Ltau) ? 0 : tau + 1;
    const uint32_t tm = (tau == 0) ? G.Ltau - 1 : tau - 1;
    const uint32_t row = y * L;
    const uint32_t plane = tau * P;

    WordState st;
    st.s = plane + row + x;
    const uint64_t w = load64<kGlobal>(S, st.s);
    const uint64_t nxp = load64<kGlobal>(S, plane + row + xp);
    const uint64_t nxm = load64<kGlobal>(S, plane + row + xm);
    const uint64_t nyp = load64<kGlobal>(S, plane + yp * L + x);
    const uint64_t nym = load64<kGlobal>(S, plane + ym * L + x);
    const uint64_t ntp_raw = load64<kGlobal>(S, tp * P + row + x);
    const uint64_t ntm_raw = load64<kGlobal>(S, tm * P + row + x);
    const uint64_t jxp = load64<true>(G.Jx, row + x);
    const uint64_t jxm = load64<true>(G.Jx, row + xm);  // the -x bond is the +x bond of x-1
    const uint64_t jyp = load64<true>(G.Jy, row + x);
    const uint64_t jym = load64<true>(G.Jy, ym * L + x);

    // unsatisfied space bonds u = w ^ neighbour ^ coupling and their count
    // n_s = s2 s1 s0: a full adder over u1..u3, then u4 added to its sum
    const uint64_t u1 = bop3<kXor3>(w, nxp, jxp), u2 = bop3<kXor3>(w, nxm, jxm);
    const uint64_t u3 = bop3<kXor3>(w, nyp, jyp), u4 = bop3<kXor3>(w, nym, jym);
    const uint64_t sum = bop3<kXor3>(u1, u2, u3), carry = bop3<kMajority>(u1, u2, u3);
    st.w = w;
    st.s0 = sum ^ u4;
    st.s1 = bop3<kXorAnd>(carry, sum, u4);
    st.s2 = bop3<kAnd3>(carry, sum, u4);
    // unsatisfied time bonds n_t as one-hot planes; on an antiperiodic prism
    // the bond that wraps round tau counts with the opposite sign, which is
    // the neighbour's word inverted
    uint64_t ntp = ntp_raw, ntm = ntm_raw;
    if (G.anti) {
        asm volatile("");  // a block-uniform branch: periodic groups skip this
        if (tau + 1 == G.Ltau) ntp = ~ntp;
        if (tau == 0) ntm = ~ntm;
    }
    st.nt0 = bop3<kEqEq>(w, ntp, ntm);
    st.nt1 = ntp ^ ntm;
    st.nt2 = bop3<kNeNe>(w, ntp, ntm);
    st.acc = 0;
    st.und = 0;
    return st;
}

// Load the neighbourhood of colour-c word `idx` of a slot and count
// unsatisfied bonds.  Colour-c words of a slot are numbered plane by plane,
// row by row: idx = tau*(L*L/2) + y*(L/2) + xh, x = 2*xh + ((c + y + tau) & 1).
template <bool kGlobal>
__device__ __forceinline__ WordState load_word(const GroupDev& G, const uint64_t* __restrict__ S,
                                               uint32_t colour, uint32_t idx) {
    const uint32_t half_plane = (G.L * G.L) >> 1;
    const uint32_t half_row = G.L >> 1;
    const uint32_t tau = fast_div(idx, G.div_half_plane);
    const uint32_t rem = idx - tau * half_plane;
    const uint32_t y = fast_div(rem, G.div_half_row);
    const uint32_t x = 2 * (rem - y * half_row) + ((colour + y + tau) & 1u);
    return load_site<kGlobal>(G, S, x, y, tau);
}

// One-hot masks of the listed classes and the slot's thresholds for them.
template <int R>
__device__ __forceinline__ void class_masks(const WordState& st, const uint32_t* __restrict__ thr,
                                            uint64_t (&M)[Classes<R>::n],
                                            uint32_t (&th)[Classes<R>::n]) {
    using C = Classes<R>;
    const uint64_t NT[3] = {st.nt0, st.nt1, st.nt2};
    const uint64_t ns0 = bop3<kNor3>(st.s2, st.s1, st.s0);
#pragma unroll
    for (int i = 0; i < C::n; ++i) {
        th[i] = __builtin_amdgcn_readfirstlane(thr[C::ns[i] * 3 + C::nt[i]]);
        const uint64_t nt = NT[C::nt[i]];
        // n_s <= 4, so s0 & ~s1 means 1, s1 & ~s0 means 2, s1 & s0 means 3
        switch (C::ns[i]) {
            case 0: M[i] = ns0 & nt; break;
            case 1: M[i] = bop3<kAndNotAnd>(st.s0, st.s1, nt); break;
            case 2: M[i] = bop3<kAndNotAnd>(st.s1, st.s0, nt); break;
            case 3: M[i] = bop3<kAnd3>(st.s1, st.s0, nt); break;
            default: M[i] = st.s2 & nt; break;
        }
        if (R == 3) M[i] &= ~all_if(th[i] == 0xFFFFFFFFu ? 1u : 0u, 0);
    }
}


// Compare the lanes' bit-sliced Philox numbers with their class thresholds,
// most significant level first, for blocks q0 <= q < q1 while any lane of
// the wave is undecided.  Block q (counter (s, t, g<<4 | q, gid)) carries
// levels 2q and 2q+1.  Per level, on each 32-bit half, with T the plane of
// the lanes' threshold bits and W the level of the random numbers:
//   acc |= und & T & ~W   (r has 0 where thr has 1: r < thr, accepted)
//   und &= ~(T ^ W)       (still equal so far).
// Regimes 0-2 build T from the slot's level pick: a block-uniform branch per
// class skips the classes outside it, so at most three masks are combined;
// the class masks are disjoint, so T = inv ^ (xor of the picked masks), with
// inv = ~0 for a complemented pick, is exact on every lane still undecided.
// Regime 3 (any table) ORs all fifteen masks, each ANDed with its bit.
template <int R>
__device__ __forceinline__ void compare_levels(const GroupDev& G, uint32_t g, uint32_t t,
                                               uint32_t s, const uint64_t (&M)[Classes<R>::n],
                                               const uint32_t (&th)[Classes<R>::n],
                                               const uint32_t* thr, uint32_t q0,
                                               uint32_t q1, uint64_t& acc, uint64_t& und,
                                               uint32_t unchecked = 0) {
    using C = Classes<R>;
    uint32_t acc_lo = (uint32_t)acc, acc_hi = (uint32_t)(acc >> 32);
    uint32_t und_lo = (uint32_t)und, und_hi = (uint32_t)(und >> 32);
    // the slot's level picks (two bytes per block, see kLevelPicks), read
    // through the constant address space: block-uniform scalar loads (the
    // table is not written during a launch)
    typedef const uint32_t __attribute__((address_space(4)))* ConstU32;
    const ConstU32 pk = (ConstU32)(thr);
#pragma unroll 1
    for (uint32_t q = q0; q < q1; ++q) {
        // every lane of the wave decided: stop (not checked for the first
        // `unchecked` blocks, where that almost never happens; a block run
        // on decided lanes changes nothing)
        if (q >= q0 + unchecked && !__any((und_lo | und_hi) != 0)) break;
        const uint4 o = philox(make_uint4(s, t, (g << 4) | q, G.gid), G.key0, G.key1);
        const uint32_t lev_lo[2] = {o.x, o.z};
        const uint32_t lev_hi[2] = {o.y, o.w};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            uint32_t T_lo = 0, T_hi = 0;
            if (R < 3) {
                const uint32_t pick = (pk[kLevelPicks + (q >> 1)] >> (16 * (q & 1u) + 8 * h)) & 0xFFu;
                T_lo = T_hi = 0u - (pick >> 7);
#pragma unroll
                for (int i = 0; i < C::n; ++i) {
                    if (pick & (1u << i)) {
                        asm volatile("");  // keep the uniform branch: no select of both sides
                        T_lo ^= (uint32_t)M[i];
                        T_hi ^= (uint32_t)(M[i] >> 32);
                    }
                }
            } else {
                const uint32_t bit = 31u - (2u * q + (uint32_t)h);
#pragma unroll
                for (int i = 0; i < C::n; ++i) {
                    const uint32_t B = 0u - ((th[i] >> bit) & 1u);  // block-uniform 0 or ~0
                    T_lo = BITOP3((uint32_t)M[i], B, T_lo, kAndOr);
                    T_hi = BITOP3((uint32_t)(M[i] >> 32), B, T_hi, kAndOr);
                }
            }
            acc_lo |= BITOP3(und_lo, T_lo, lev_lo[h], kAndAndNot);
            acc_hi |= BITOP3(und_hi, T_hi, lev_hi[h], kAndAndNot);
            und_lo = BITOP3(und_lo, T_lo, lev_lo[h], kAndXnor);
            und_hi = BITOP3(und_hi, T_hi, lev_hi[h], kAndXnor);
        }
    }
    acc = lo_hi(acc_lo, acc_hi);
    und = lo_hi(und_lo, und_hi);
}

__device__ __forceinline__ void put_slot(SweepQueue& Q, uint32_t o, const WordState& st) {
    Q.s[o] = st.s;
    Q.w[o] = st.w;
    Q.s0[o] = st.s0;
    Q.s1[o] = st.s1;
    Q.s2[o] = st.s2;
    Q.nt0[o] = st.nt0;
    Q.nt2[o] = st.nt2;
}

__device__ __forceinline__ void push_word(SweepQueue& Q, uint32_t k, uint32_t owner, uint64_t acc,
                                          uint64_t und) {
    Q.owner[k] = owner;
    Q.acc[k] = acc;
    Q.und[k] = und;
}

// Entry k of the queue with its owner's slot.
__device__ __forceinline__ WordState pop_word(const SweepQueue& Q, uint32_t k, uint32_t& owner) {
    WordState r;
    const uint32_t o = Q.owner[k];
    owner = o;
    r.s = Q.s[o];
    r.w = Q.w[o];
    r.s0 = Q.s0[o];
    r.s1 = Q.s1[o];
    r.s2 = Q.s2[o];
    r.nt0 = Q.nt0[o];
    r.nt2 = Q.nt2[o];
    r.nt1 = ~(r.nt0 | r.nt2);
    r.acc = Q.acc[k];
    r.und = Q.und[k];
    return r;
}

// The comparison of one word from level block q to the end (16 blocks, all
// 32 bits), then its update.
template <int R, bool kGlobal>
__device__ __forceinline__ void finish_word(const GroupDev& G, uint64_t* __restrict__ S, uint32_t g,
                                            uint32_t t, WordState r, uint32_t q) {
    using C = Classes<R>;
    const uint32_t* __restrict__ thr = G.thr + g * kThrStride;
    uint64_t M[C::n];
    uint32_t th[C::n];
    class_masks<R>(r, thr, M, th);
    compare_levels<R>(G, g, t, r.s, M, th, thr, q, 16, r.acc, r.und);
    r.acc |= r.und;  // equal on all 32 bits: r == thr, accepted
    if (r.acc) store64<kGlobal>(S, r.s, r.w ^ r.acc);
}

// The colour-pass update of one word per thread of the block: the first
// q_split Philox blocks of levels for every word; then, while the words with
// undecided lanes fill more than one wave, they are packed into the first
// waves of the block and given one more block; the last ones (at most one
// wave) are finished there.  Far fewer waves run the long tail of levels.
// Every thread of the block calls this (it synchronises); `valid` is false
// for threads without a word (st is then unused).  Packing counters: one
// pair per call parity (see SweepQueue); within a call, round j writes
// counter j & 1, which round j - 1 cleared after every thread had read its
// previous value.
template <int R, bool kGlobal>
__device__ __forceinline__ void sweep_words(const GroupDev& G, uint64_t* __restrict__ S, uint32_t g,
                                            uint32_t t, WordState st, bool valid, uint32_t q_split,
                                            SweepQueue& Q, uint32_t parity) {
    using C = Classes<R>;
    const uint32_t* __restrict__ thr = G.thr + g * kThrStride;
    uint32_t* cnt = Q.count + 2 * (parity & 1u);
    if (threadIdx.x == 0) {
        cnt[0] = 0;
        cnt[1] = 0;
    }
    __syncthreads();
    uint64_t M[C::n];
    uint32_t th[C::n];
    if (valid) {
        put_slot(Q, threadIdx.x, st);
        class_masks<R>(st, thr, M, th);
        uint64_t live = 0;
#pragma unroll
        for (int i = 0; i < C::n; ++i) live |= M[i];
        st.acc = ~live;  // lanes outside the listed classes: dE <= 0, accepted
        st.und = live;
        compare_levels<R>(G, g, t, st.s, M, th, thr, 0, q_split, st.acc, st.und, 0);
        if (st.und != 0)
            push_word(Q, atomicAdd(&cnt[0], 1u), threadIdx.x, st.acc, st.und);
        else if (st.acc)
            store64<kGlobal>(S, st.s, st.w ^ st.acc);
    }
    __syncthreads();
    uint32_t n = __builtin_amdgcn_readfirstlane(cnt[0]);
    uint32_t q = q_split;
#pragma unroll 1
    for (uint32_t j = 1; n > kWaveSize && q + 1 < 16; ++j, ++q) {
        const bool have = threadIdx.x < n;
        WordState r;
        uint32_t owner = 0;
        if (have) r = pop_word(Q, threadIdx.x, owner);
        __syncthreads();  // every entry and count read before any is rewritten
        if (threadIdx.x == 0) cnt[(j + 1) & 1u] = 0;
        if (have) {
            class_masks<R>(r, thr, M, th);
            compare_levels<R>(G, g, t, r.s, M, th, thr, q, q + 1, r.acc, r.und);
            if (r.und != 0)
                push_word(Q, atomicAdd(&cnt[j & 1u], 1u), owner, r.acc, r.und);
            else if (r.acc)
                store64<kGlobal>(S, r.s, r.w ^ r.acc);
        }
        __syncthreads();
        n = __builtin_amdgcn_readfirstlane(cnt[j & 1u]);
    }
    // the last words are finished where they sit in the queue
    if (threadIdx.x < n) {
        uint32_t owner;
        finish_word<R, kGlobal>(G, S, g, t, pop_word(Q, threadIdx.x, owner), q);
    }
}

// One word per thread, numbered as in load_word (the fused chunk kernel).
template <int R, bool kGlobal>
__device__ __forceinline__ void sweep_block(const GroupDev& G, uint64_t* __restrict__ S, uint32_t g,
                                            uint32_t colour, uint32_t t, uint32_t idx, bool valid,
                                            uint32_t q_split, SweepQueue& Q, uint32_t parity) {
    WordState st{};
    if (valid) st = load_word<kGlobal>(G, S, colour, idx);
    sweep_words<R, kGlobal>(G, S, g, t, st, valid, q_split, Q, parity);
}

// Column walk: thread `item` of a slot owns column (x, y) = item mod L^2 of
// tau tile item / L^2 (G.tile planes, tile * G.tile ... + G.tile - 1); its
// colour-c sites there are tau = tau0 + par, tau0 + par + 2, ..., with
// par = (c + x + y) & 1, one per step.  Offsets of the centre and its four
// space neighbours are fixed for the walk and the slot base advances by two
// planes per step (a block-uniform address on the scalar unit), the four
// couplings are loaded once, and the word below the centre is the previous
// step's word above it, so a step costs six loads and no index arithmetic.
// Only the first step's lower neighbour and the last step's upper one can
// wrap round tau.
__device__ __forceinline__ uint64_t load_at(const uint64_t* base, uint32_t byte_off) {
    return *(const uint64_t __attribute__((address_space(1)))*)((const GlobalByte*)base + byte_off);
}

// A block-uniform pointer read back through the scalar unit: the compiler
// then forms each address as this scalar base plus a 32-bit offset inside
// the loop instead of keeping 64-bit per-thread addresses live across it.
template <typename T>
__device__ __forceinline__ T* scalar_ptr(T* p) {
    const uint64_t v = (uint64_t)(uintptr_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (T*)(uintptr_t)lo_hi(lo, hi);
}

template <int R>
__device__ __forceinline__ void walk_block(const GroupDev& G, uint64_t* __restrict__ S, uint32_t g,
                                           uint32_t colour, uint32_t t, uint32_t item, bool valid,
                                           SweepQueue& Q) {
    const uint32_t L = G.L, P = L * L, Ltau = G.Ltau;
    const uint32_t steps = G.tile >> 1;
    uint32_t tile = 0, col = 0;
    if (valid) {
        tile = fast_div(item, G.div_plane);
        col = item - tile * P;
    }
    const uint32_t y = fast_div(col, G.div_row);
    const uint32_t x = col - y * L;
    const uint32_t xp = (x + 1 == L) ? 0 : x + 1;
    const uint32_t xm = (x == 0) ? L - 1 : x - 1;
    const uint32_t yp = (y + 1 == L) ? 0 : y + 1;
    const uint32_t ym = (y == 0) ? L - 1 : y - 1;
    const uint32_t row = y * L;
    const uint32_t tau0 = tile * G.tile + ((colour + x + y) & 1u);
    const uint32_t plane0 = tau0 * P;
    // byte offsets from the step's base S + 2 k P (k = step)
    uint32_t o_c = (plane0 + row + x) * 8u;
    uint32_t o_xp = (plane0 + row + xp) * 8u, o_xm = (plane0 + row + xm) * 8u;
    uint32_t o_yp = (plane0 + yp * L + x) * 8u, o_ym = (plane0 + ym * L + x) * 8u;
    uint32_t o_tp = o_c + P * 8u;
    // coupling words, reloaded every step (cache hits) rather than held
    uint32_t j_c = (row + x) * 8u, j_xm = (row + xm) * 8u, j_ym = (ym * L + x) * 8u;
    uint64_t below = 0;
    if (valid) {
        if (tau0 == 0) {  // the bond round tau: slice Ltau-1, sign flipped if antiperiodic
            below = load64<true>(S, (Ltau - 1) * P + row + x);
            if (G.anti) below = ~below;
        } else {
            below = load_at(S, o_c - P * 8u);
        }
    }
    const uint32_t site0 = plane0 + row + x;
    const uint64_t* S0 = scalar_ptr(S);
    const uint64_t* Jx = scalar_ptr(G.Jx);
    const uint64_t* Jy = scalar_ptr(G.Jy);
#pragma unroll 1
    for (uint32_t k = 0; k < steps; ++k) {
        const uint64_t* Sk = S0 + (size_t)k * 2 * P;
        // the offsets stay 32-bit values in the loop (scalar base + 32-bit
        // offset addressing), not 64-bit addresses hoisted out of it
        asm volatile("" : "+v"(o_c), "+v"(o_xp), "+v"(o_xm), "+v"(o_yp), "+v"(o_ym), "+v"(o_tp));
        asm volatile("" : "+v"(j_c), "+v"(j_xm), "+v"(j_ym));
        WordState st;
        if (valid) {
            const uint64_t w = load_at(Sk, o_c);
            const uint64_t nxp = load_at(Sk, o_xp), nxm = load_at(Sk, o_xm);
            const uint64_t nyp = load_at(Sk, o_yp), nym = load_at(Sk, o_ym);
            uint64_t above;
            if (k + 1 == steps && tau0 + 2 * k + 1 == Ltau) {  // top slice: wraps to slice 0
                above = load64<true>(S, row + x);
                if (G.anti) above = ~above;
            } else {
                above = load_at(Sk, o_tp);
            }
            st.s = site0 + 2 * k * P;
            const uint64_t jxp = load_at(Jx, j_c);
            const uint64_t jxm = load_at(Jx, j_xm);  // the -x bond is the +x bond of x-1
            const uint64_t jyp = load_at(Jy, j_c);
            const uint64_t jym = load_at(Jy, j_ym);
            const uint64_t u1 = bop3<kXor3>(w, nxp, jxp), u2 = bop3<kXor3>(w, nxm, jxm);
            const uint64_t u3 = bop3<kXor3>(w, nyp, jyp), u4 = bop3<kXor3>(w, nym, jym);
            const uint64_t sum = bop3<kXor3>(u1, u2, u3), carry = bop3<kMajority>(u1, u2, u3);
            st.w = w;
            st.s0 = sum ^ u4;
            st.s1 = bop3<kXorAnd>(carry, sum, u4);
            st.s2 = bop3<kAnd3>(carry, sum, u4);
            st.nt0 = bop3<kEqEq>(w, above, below);
            st.nt1 = above ^ below;
            st.nt2 = bop3<kNeNe>(w, above, below);
            below = above;
        }
        sweep_words<R, true>(G, S, g, t, st, valid, G.q_split, Q, k);
    }
}
// S: the slot's spins (global memory, or a copy in LDS).
// parity: alternate 0/1 between consecutive calls in one block.
template <bool kGlobal>
__device__ __forceinline__ void sweep_block_any(const GroupDev& G, uint64_t* S, uint32_t g,
                                                uint32_t colour, uint32_t t, uint32_t idx,
                                                bool valid, uint32_t q_split, SweepQueue& Q,
                                                uint32_t parity) {
    switch (__builtin_amdgcn_readfirstlane(G.thr[g * kThrStride + 15])) {  // slot g's regime
        case 0: sweep_block<0, kGlobal>(G, S, g, colour, t, idx, valid, q_split, Q, parity); break;
        case 1: sweep_block<1, kGlobal>(G, S, g, colour, t, idx, valid, q_split, Q, parity); break;
        case 2: sweep_block<2, kGlobal>(G, S, g, colour, t, idx, valid, q_split, Q, parity); break;
        default: sweep_block<3, kGlobal>(G, S, g, colour, t, idx, valid, q_split, Q, parity); break;
    }
}

// Slots whose tables fit none of the three seven-class regimes (never the
// case for the tables of either ladder kind, whose couplings are positive)
// take the fifteen-class update one word per thread, without the walk's
// registers: thread `item` updates colour-c words item, item + n, ... with
// n = V / tile threads per slot.
__device__ __forceinline__ void walk_block_any(const GroupDev& G, uint64_t* S, uint32_t g,
                                               uint32_t colour, uint32_t t, uint32_t item,
                                               uint32_t n_items, SweepQueue& Q) {
    const bool valid = item < n_items;
    switch (__builtin_amdgcn_readfirstlane(G.thr[g * kThrStride + 15])) {  // slot g's regime
        case 0: walk_block<0>(G, S, g, colour, t, item, valid, Q); break;
        case 1: walk_block<1>(G, S, g, colour, t, item, valid, Q); break;
        case 2: walk_block<2>(G, S, g, colour, t, item, valid, Q); break;
        default:
#pragma unroll 1
            for (uint32_t k = 0; k < (G.tile >> 1); ++k)
                sweep_block<3, true>(G, S, g, colour, t, item + k * n_items, valid, G.q_split, Q, k);
            break;
    }
}

// Blocks are dealt to the eight XCDs round-robin (block b runs on XCD b % 8).
// Renumber them so that every XCD receives one contiguous run of logical
// blocks: neighbouring tau-planes then meet in the same L2.  A bijection of
// [0, n); only the speed depends on the dispatch order.
__device__ __forceinline__ uint32_t xcd_contiguous(uint32_t b, uint32_t n) {
    constexpr uint32_t kXcd = 8;
    const uint32_t q = n / kXcd, r = n % kXcd;
    const uint32_t x = b % kXcd, i = b / kXcd;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

__global__ void __launch_bounds__(kSweepBlock)
k_half_sweep(const GroupDev G, uint32_t colour, const uint32_t* __restrict__ ctr, uint32_t t_add) {
    __shared__ SweepQueue Q;
    const uint32_t t = __builtin_amdgcn_readfirstlane(ctr[0] + t_add);
    const uint32_t b = xcd_contiguous(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
    const uint32_t g = fast_div(b, G.div_blocks);  // b / gridDim.x on the scalar unit
    const uint32_t item = (b - g * gridDim.x) * kSweepBlock + threadIdx.x;
    walk_block_any(G, G.spins + (size_t)g * G.V, g, colour, t, item, G.V >> __builtin_ctz(G.tile), Q);
}

__device__ __forceinline__ uint32_t find_group(const uint32_t* __restrict__ prefix,
                                               uint32_t n_groups, uint32_t b) {
    uint32_t lo = 0, hi = n_groups;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (prefix[mid] <= b) lo = mid; else hi = mid;
    }
    return lo;
}

// Record of group gi.  For groups of one shape (kSameShape: the plan's
// same_shape, chosen at launch so that each instantiation has one path) it
// is the kernel argument's copy with the pointers moved to group gi and the
// group's own Philox identity: no load stands between the block's start and
// its first address computation (the three identity words are needed only
// later).  Otherwise the record is read from memory.
template <typename T>
__device__ __forceinline__ T* advance(T* p, uint64_t bytes) {
    return (T*)((char*)p + bytes);
}
template <bool kSameShape>
__device__ __forceinline__ GroupDev group_record(const BatchPlan& p, uint32_t gi) {
    if (!kSameShape) return uniform_record(p.groups + gi);
    GroupDev G = p.first;
    const uint64_t d = (uint64_t)gi * p.stride;
    G.spins = advance(G.spins, d);
    G.Jx = advance(G.Jx, d);
    G.Jy = advance(G.Jy, d);
    G.jseed = advance(G.jseed, d);
    G.thr = advance(G.thr, d);
    G.sw_thr = advance(G.sw_thr, d);
    G.sw_len = advance(G.sw_len, d);
    G.sw_eq = advance(G.sw_eq, d);
    G.cnt = advance(G.cnt, d);
    G.E = advance(G.E, d);
    G.walker = advance(G.walker, d);
    G.rt = advance(G.rt, d);
    G.acc = advance(G.acc, d);
    G.swaplog = advance(G.swaplog, d);
    G.sums = advance(G.sums, d);
    G.lastmask = advance(G.lastmask, d);
    G.meas = advance(G.meas, d);
    G.hist = advance(G.hist, d);
    const GroupDev* __restrict__ r = p.groups + gi;
    G.gid = __builtin_amdgcn_readfirstlane(r->gid);
    G.key0 = __builtin_amdgcn_readfirstlane(r->key0);
    G.key1 = __builtin_amdgcn_readfirstlane(r->key1);
    return G;
}

// Group of block b of a batched launch and the block's index within that
// group.  Groups of one size (the usual ensemble) take one scalar division;
// otherwise one load from the plan's block map where it has one, else a
// binary search of the prefix sums (a chain of dependent scalar loads that
// delays every block's first spin load).  kSameShape: the plan's groups
// share one shape, so they have equal block counts and only the division is
// compiled in.
struct BlockPlace {
    uint32_t gi, local;
};
template <bool kSameShape>
__device__ __forceinline__ BlockPlace locate(const BatchPlan& p, uint32_t b) {
    if (kSameShape || p.per_group) {
        const uint32_t gi = fast_div(b, p.span);
        return {gi, b - gi * p.per_group};
    }
    if (p.block_map) {
        const BlockEntry e = p.block_map[b];
        return {(uint32_t)__builtin_amdgcn_readfirstlane(e.gi),
                (uint32_t)__builtin_amdgcn_readfirstlane(e.local)};
    }
    const uint32_t gi = find_group(p.prefix, p.n_groups, b);
    return {gi, b - p.prefix[gi]};
}

template <bool kSameShape>
__global__ void __launch_bounds__(kSweepBlock)
k_half_sweep_batched(const BatchPlan plan, uint32_t colour, const uint32_t* __restrict__ ctr,
                     uint32_t t_add) {
    __shared__ SweepQueue Q;
    const uint32_t t = __builtin_amdgcn_readfirstlane(ctr[0] + t_add);
    const uint32_t b = xcd_contiguous(blockIdx.x, gridDim.x);
    const BlockPlace at = locate<kSameShape>(plan, b);
    const GroupDev G = group_record<kSameShape>(plan, at.gi);
    const uint32_t local = __builtin_amdgcn_readfirstlane(at.local);
    const uint32_t nb = sweep_blocks_per_slot(G.V, G.tile);
    const uint32_t g = fast_div(local, G.div_blocks);  // local / nb on the scalar unit
    const uint32_t item = (local - g * nb) * kSweepBlock + threadIdx.x;
    walk_block_any(G, G.spins + (size_t)g * G.V, g, colour, t, item, G.V >> __builtin_ctz(G.tile), Q);
}

// ---------------------------------------------------------------------------
// Fused sweeps: one block owns one slot for `n_sweeps` sweeps (no other
// block touches it before the PT step), so colour passes are separated by
// block barriers only and all sweeps of a PT chunk are one launch.  Slots of
// at most `lds_words` words are copied into LDS for the chunk.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kSweepBlock)
k_chunk_fused(const BatchPlan slots, const uint32_t* __restrict__ ctr, uint32_t n_sweeps,
              uint32_t lds_words) {
    extern __shared__ uint64_t lds_spins[];
    __shared__ SweepQueue Q;
    const BlockPlace at = locate<false>(slots, blockIdx.x);
    const GroupDev G = group_record<false>(slots, at.gi);
    const uint32_t g = __builtin_amdgcn_readfirstlane(at.local);
    const uint32_t V = G.V, half = V >> 1;
    uint64_t* Sg = G.spins + (size_t)g * V;
    const bool in_lds = V <= lds_words;
    uint64_t* S = in_lds ? lds_spins : Sg;
    if (in_lds) {
        for (uint32_t i = threadIdx.x; i < V; i += kSweepBlock) lds_spins[i] = Sg[i];
        __syncthreads();
    }
    const uint32_t t0 = __builtin_amdgcn_readfirstlane(ctr[0]);
    uint32_t call = 0;
    for (uint32_t it = 0; it < n_sweeps; ++it) {
        for (uint32_t colour = 0; colour < 2; ++colour) {
            for (uint32_t base = 0; base < half; base += kSweepBlock) {
                const uint32_t idx = base + threadIdx.x;
                sweep_block_any<false>(G, S, g, colour, t0 + it, idx, idx < half, G.q_split, Q, call++);
            }
            __syncthreads();  // the next colour reads what this one wrote
        }
    }
    if (in_lds)
        for (uint32_t i = threadIdx.x; i < V; i += kSweepBlock) Sg[i] = lds_spins[i];
}

// ---------------------------------------------------------------------------
// Energy / overlap pass: per slot and lane, the number of unsatisfied space
// bonds and time bonds (each bond counted once, from its lower endpoint),
// and per lane pair (2p, 2p+1) the number of sites where they differ.
// Each thread adds its words into bit-sliced vertical counters; each wave
// then turns counters into per-lane totals (a bit transpose across the wave
// and popcounts) and adds them to the slot's counters with integer atomics
// (order-independent, exact).
// ---------------------------------------------------------------------------
// Bit-sliced per-lane counter: value = ones + 2 twos + 4 fours + 8 * (hi as
// a binary number).  Planes are added four at a time with carry-save adders
// (Harley-Seal): three adders, then the carry into `fours` and the binary
// part rippled once per four planes.
// Binary planes a LaneCounter needs above ones/twos/fours to hold `max`.
constexpr int counter_planes(int max) {
    int nh = 0;
    while ((8 << nh) - 1 < max) ++nh;
    return nh;
}

template <int NH>
struct LaneCounter {
    uint64_t ones = 0, twos = 0, fours = 0;
    uint64_t hi[NH] = {};
};

// carry-save adder: (h, l) with a + b + c = 2h + l per lane
__device__ __forceinline__ void csa(uint64_t& h, uint64_t& l, uint64_t a, uint64_t b, uint64_t c) {
    const uint32_t alo = (uint32_t)a, blo = (uint32_t)b, clo = (uint32_t)c;
    const uint32_t ahi = (uint32_t)(a >> 32), bhi = (uint32_t)(b >> 32), chi = (uint32_t)(c >> 32);
    l = lo_hi(__builtin_amdgcn_bitop3_b32(alo, blo, clo, 0x96),
              __builtin_amdgcn_bitop3_b32(ahi, bhi, chi, 0x96));  // a ^ b ^ c
    h = lo_hi(__builtin_amdgcn_bitop3_b32(alo, blo, clo, 0xE8),
              __builtin_amdgcn_bitop3_b32(ahi, bhi, chi, 0xE8));  // majority
}

template <int NH>
__device__ __forceinline__ void add4(LaneCounter<NH>& c, const uint64_t (&x)[4]) {
    uint64_t twosA, twosB, fours;
    csa(twosA, c.ones, c.ones, x[0], x[1]);
    csa(twosB, c.ones, c.ones, x[2], x[3]);
    csa(fours, c.twos, c.twos, twosA, twosB);
    uint64_t eights = c.fours & fours;
    c.fours ^= fours;
#pragma unroll
    for (int i = 0; i < NH; ++i) {
        const uint64_t carry = c.hi[i] & eights;
        c.hi[i] ^= eights;
        eights = carry;
    }
}

// 64 x 64 bit transpose across the wave: afterwards thread t holds, in bit
// b, bit t of thread b's word.  Stage k exchanges with thread t ^ 2^k the
// bits whose index differs from t in bit k (swapping bit k of the thread
// index with bit k of the bit index); the six stages commute.  Stage 5
// swaps the roles of the two 32-bit halves: a thread sends its partner the
// half the partner keeps and takes one half back.  Stages 0-4 stay inside
// each half: a thread keeps its bits on one side of bit k (mask K) and takes
// the partner's other side, rotated into place by one v_alignbit (right by
// 2^k if it keeps the upper side, else by 32 - 2^k), then one v_bitop3
// merges the two.
__device__ __forceinline__ uint64_t wave_transpose(uint64_t x) {
    const uint32_t t = threadIdx.x & 63u;
    uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
    {
        const bool up = (t & 32u) != 0;
        const uint32_t recv = (uint32_t)__shfl_xor((int)(up ? lo : hi), 32, 64);
        lo = up ? recv : lo;
        hi = up ? hi : recv;
    }
    constexpr uint32_t kHigh[5] = {0xAAAAAAAAu, 0xCCCCCCCCu, 0xF0F0F0F0u, 0xFF00FF00u, 0xFFFF0000u};
#pragma unroll
    for (int k = 4; k >= 0; --k) {
        const uint32_t sh = 1u << k;
        const bool up = (t & sh) != 0;
        const uint32_t keep = up ? kHigh[k] : ~kHigh[k];
        const uint32_t rot = up ? sh : 32u - sh;
        const uint32_t ylo = (uint32_t)__shfl_xor((int)lo, (int)sh, 64);
        const uint32_t yhi = (uint32_t)__shfl_xor((int)hi, (int)sh, 64);
        lo = BITOP3(keep, lo, __builtin_amdgcn_alignbit(ylo, ylo, rot), kSelect);
        hi = BITOP3(keep, hi, __builtin_amdgcn_alignbit(yhi, yhi, rot), kSelect);
    }
    return lo_hi(lo, hi);
}

// Per-lane totals over the wave's 64 threads of a bit-sliced counter: thread
// t gets the total of lane t.
template <int NH>
__device__ __forceinline__ uint32_t lane_total(const LaneCounter<NH>& c) {
    uint32_t tot = (uint32_t)__popcll(wave_transpose(c.ones)) +
                   ((uint32_t)__popcll(wave_transpose(c.twos)) << 1) +
                   ((uint32_t)__popcll(wave_transpose(c.fours)) << 2);
#pragma unroll
    for (int i = 0; i < NH; ++i) tot += (uint32_t)__popcll(wave_transpose(c.hi[i])) << (3 + i);
    return tot;
}

// Column walk: thread `item` of slot g owns column (x, y) = item mod L^2 of
// tau tile item / L^2 (`planes` planes, planes dividing Ltau) and walks it
// bottom to top.  Each bond is counted once, from its lower endpoint: per
// word the +x and +y neighbours in the same plane and the word above, which
// is the next step's centre, so a step costs three loads; the offsets are
// fixed for the walk and the slot base advances one plane per step.  Only
// the tile's last bond can wrap round tau.
//
// The walk runs in batches of kEnergyBatch steps, software-pipelined: the
// loads of the next batch are issued before the current batch is counted,
// so every wave keeps loads in flight while it adds.  For that the loads of
// a batch take no branch (the compiler would otherwise wait for every load
// in flight before counting): steps past the tile's end re-read its last
// plane and are not counted, the wrapping bond's word comes through a
// selected offset, and its antiperiodic sign is applied when counting.
constexpr int kEnergyBatch = 4;

struct EnergyBatch {
    uint64_t up[kEnergyBatch], xp[kEnergyBatch], yp[kEnergyBatch];
};

template <int kMaxPlanes>
__device__ __forceinline__ void energy_walk(const GroupDev& G, uint32_t g, uint32_t item,
                                            uint32_t planes, int32_t* __restrict__ cnt) {
    const uint32_t L = G.L, P = L * L;
    const uint32_t n_items = G.V >> __builtin_ctz(planes);
    // a wave without a column (the tail of a slot's last block) has nothing
    // to add: it leaves before the cross-lane transposes
    if (__builtin_amdgcn_readfirstlane(item) >= n_items) return;
    const uint64_t* __restrict__ S = G.spins + (size_t)g * G.V;
    // per thread and lane at most 2*kMaxPlanes unsatisfied space bonds and
    // kMaxPlanes time bonds or differing pairs
    LaneCounter<counter_planes(2 * kMaxPlanes)> Csp;
    LaneCounter<counter_planes(kMaxPlanes)> Ct, Cq;
    if (item < n_items) {
        const uint32_t tile = fast_div(item, G.div_plane);
        const uint32_t col = item - tile * P;
        const uint32_t y = fast_div(col, G.div_row);
        const uint32_t x = col - y * L;
        const uint32_t xp = (x + 1 == L) ? 0 : x + 1;
        const uint32_t yp = (y + 1 == L) ? 0 : y + 1;
        const uint32_t base = tile * planes * P;
        // byte offsets: o_xp, o_yp from the step's plane; up words from S
        uint32_t o_xp = (base + y * L + xp) * 8u, o_yp = (base + yp * L + x) * 8u;
        uint32_t o_up = (base + col + P) * 8u;
        const uint32_t o_wrap = col * 8u;  // slice 0, above the top slice
        const uint64_t jx = G.Jx[col], jy = G.Jy[col];
        const bool top = tile * planes + planes == G.Ltau;  // the last bond wraps to slice 0
        const uint64_t flip = (top && G.anti) ? ~0ull : 0ull;  // antiperiodic wrap bond
        const uint32_t last = planes - 1;
        auto fetch = [&](uint32_t k0, EnergyBatch& B) {
            asm volatile("" : "+v"(o_up), "+v"(o_xp), "+v"(o_yp));  // 32-bit offsets in the loop
#pragma unroll
            for (int k = 0; k < kEnergyBatch; ++k) {
                const uint32_t kk = min(k0 + k, last);  // block-uniform
                const uint64_t* Sk = scalar_ptr(S + (size_t)kk * P);
                B.xp[k] = load_at(Sk, o_xp);
                B.yp[k] = load_at(Sk, o_yp);
                B.up[k] = load_at(S, (top && kk == last) ? o_wrap : o_up + kk * P * 8u);
            }
        };
        uint64_t w = load_at(S, (base + col) * 8u);
        // kGuard: some steps of the batch may lie past the tile's end
        auto count = [&](auto guard, uint32_t k0, const EnergyBatch& B) {
            constexpr bool kGuard = decltype(guard)::value;
            uint64_t xs[kEnergyBatch], ys[kEnergyBatch], ts[kEnergyBatch], qs[kEnergyBatch];
#pragma unroll
            for (int k = 0; k < kEnergyBatch; ++k) {
                xs[k] = ys[k] = ts[k] = qs[k] = 0;
                if (!kGuard || k0 + k < planes) {  // block-uniform
                    const uint64_t up = B.up[k];
                    xs[k] = bop3<kXor3>(w, B.xp[k], jx);  // +x bond unsatisfied
                    ys[k] = bop3<kXor3>(w, B.yp[k], jy);  // +y bond unsatisfied
                    ts[k] = bop3<kXor3>(w, up, k0 + k == last ? flip : 0ull);  // +tau bond
                    // pair (2p, 2p+1) differs; pairs never straddle the halves
                    const uint32_t lo = (uint32_t)w, hi = (uint32_t)(w >> 32);
                    qs[k] = lo_hi(BITOP3(lo, lo >> 1, 0x55555555u, 0x28),
                                  BITOP3(hi, hi >> 1, 0x55555555u, 0x28));
                    w = up;
                }
            }
            add4(Csp, xs);
            add4(Csp, ys);
            add4(Ct, ts);
            add4(Cq, qs);
        };
        EnergyBatch b0, b1;
        if (planes % (2 * kEnergyBatch) == 0) {
            // two batch buffers used in turn (no copies between them); the
            // last fetch re-reads the top plane and is not counted
            fetch(0, b0);
#pragma unroll 1
            for (uint32_t k0 = 0; k0 < planes; k0 += 2 * kEnergyBatch) {
                fetch(k0 + kEnergyBatch, b1);
                count(std::false_type{}, k0, b0);
                fetch(k0 + 2 * kEnergyBatch, b0);
                count(std::false_type{}, k0 + kEnergyBatch, b1);
            }
        } else {  // tiles of 2 or 4 planes
#pragma unroll 1
            for (uint32_t k0 = 0; k0 < planes; k0 += kEnergyBatch) {
                fetch(k0, b0);
                count(std::true_type{}, k0, b0);
            }
        }
    }
    // every thread of the wave takes part in the transposes
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t my_sp = lane_total(Csp), my_t = lane_total(Ct);
    const uint32_t my_q = lane_total(Cq);  // pair p's total sits at lane 2p
    int32_t* __restrict__ c = cnt + g * kCntStride;
    if (my_sp) atomicAdd(&c[lane], (int32_t)my_sp);
    if (my_t) atomicAdd(&c[64 + lane], (int32_t)my_t);
    if (!(lane & 1u) && my_q) atomicAdd(&c[128 + (lane >> 1)], (int32_t)my_q);
}

__global__ void __launch_bounds__(kEnergyBlock)
k_energy(const GroupDev G, int32_t* cnt, uint32_t planes) {
    energy_walk<kEnergyPlanesSlot>(G, blockIdx.y, blockIdx.x * kEnergyBlock + threadIdx.x, planes,
                                   cnt);
}

__global__ void __launch_bounds__(kEnergyBlock)
k_energy_batched(const BatchPlan plan) {
    const BlockPlace at = locate<false>(plan, blockIdx.x);
    const GroupDev G = group_record<false>(plan, at.gi);
    const uint32_t local = at.local;
    const uint32_t nb = energy_blocks_per_slot(G.V, G.etile);
    // block-uniform: keeps the slot's address arithmetic on the scalar unit
    const uint32_t g = __builtin_amdgcn_readfirstlane(local / nb);
    energy_walk<kEnergyWords>(G, g, (local - g * nb) * kEnergyBlock + threadIdx.x, G.etile, G.cnt);
}

// ---------------------------------------------------------------------------
// Parallel tempering step of one group: 64 threads, thread j = lane j.
// Turns the pass counters into bond sums, accumulates the measurement sums,
// then visits pairs g = 0..N-2 in order; `cur` is the configuration that
// currently sits at slot g (it may have arrived from g-1 in this step).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void pt_group(const GroupDev& G, uint32_t p) {
    // The pass's energies and the walker labels of this group, lane j's
    // column of each: the pairs are visited in order, each seeing the state
    // the previous one left, so the chain runs on LDS instead of on global
    // loads.  One wave per group: no barriers needed.
    __shared__ int32_t s_sp[kMaxSlots][64], s_t[kMaxSlots][64];
    __shared__ uint32_t s_w[kMaxSlots][64];
    __shared__ uint64_t s_mask[kMaxSlots];
    const uint32_t j = threadIdx.x;
    const uint32_t N = G.N;
    const int32_t V = (int32_t)G.V;
    for (uint32_t g = 0; g < N; ++g) {
        int32_t* c = G.cnt + g * kCntStride;
        const int32_t bsp = 2 * V - 2 * c[j];
        const int32_t bt = V - 2 * c[64 + j];
        c[j] = 0;
        c[64 + j] = 0;
        s_sp[g][j] = bsp;
        s_t[g][j] = bt;
        s_w[g][j] = G.walker[g * 64 + j];
        int64_t* sm = G.sums + (size_t)g * kSumStride;
        sm[j] += bsp;
        sm[64 + j] += bt;
        const uint32_t u = (uint32_t)(V - bt) >> 1;
        atomicAdd(&G.hist[g * kHistBins + (uint32_t)(((uint64_t)u * kHistBins) / ((uint64_t)V + 1))], 1u);
        if (j < 32) {
            const int64_t q = (int64_t)V - 2 * (int64_t)c[128 + j];
            c[128 + j] = 0;
            sm[128 + j] += q;
            sm[160 + j] += q * q;
        }
    }
    int32_t cur_sp = s_sp[0][j], cur_t = s_t[0][j];
    uint32_t cur_w = s_w[0][j];
    // per-pair table lengths and equal-slot flags, lane g holding pair g's
    const uint32_t my_len = j + 1 < N ? G.sw_len[j] : 0u;
    const uint32_t my_eq = j + 1 < N ? (uint32_t)G.sw_eq[j] : 0u;
    uint64_t any = 0;
    for (uint32_t g = 0; g + 1 < N; ++g) {
        const int32_t nx_sp = s_sp[g + 1][j];
        const int32_t nx_t = s_t[g + 1][j];
        const uint32_t nx_w = s_w[g + 1][j];
        // |Bsp| <= 2V and |Bt| <= V with V <= 2^29: the difference of two
        // whole energies needs 64 bits, that of two time-bond sums does not
        const int64_t D = G.exch_all ? ((int64_t)nx_sp + nx_t) - ((int64_t)cur_sp + cur_t)
                                     : (int64_t)(nx_t - cur_t);
        bool accept;
        const uint32_t len = __builtin_amdgcn_readlane(my_len, g);
        if (__builtin_amdgcn_readlane(my_eq, g) || D >= 0) {
            accept = true;
        } else {
            const uint32_t m = (uint32_t)((uint64_t)(-D) >> 2);
            const uint32_t th = (m >= 1 && m <= len) ? G.sw_thr[(size_t)g * G.sw_cap + (m - 1)] : 0u;
            const uint4 o = philox(make_uint4(j >> 2, p, (1u << 24) | g, G.gid), G.key0, G.key1);
            const uint32_t sel = j & 3u;
            const uint32_t r = sel == 0 ? o.x : sel == 1 ? o.y : sel == 2 ? o.z : o.w;
            accept = r <= th;
        }
        const uint64_t mask = __ballot((int)accept);
        if (accept) {  // slot g takes the next configuration; cur moves up
            s_sp[g][j] = nx_sp;
            s_t[g][j] = nx_t;
            s_w[g][j] = nx_w;
        } else {       // cur stays at g; the next one becomes cur
            s_sp[g][j] = cur_sp;
            s_t[g][j] = cur_t;
            s_w[g][j] = cur_w;
            cur_sp = nx_sp;
            cur_t = nx_t;
            cur_w = nx_w;
        }
        if (j == 0) s_mask[g] = mask;
        any |= mask;
    }
    s_sp[N - 1][j] = cur_sp;
    s_t[N - 1][j] = cur_t;
    s_w[N - 1][j] = cur_w;
    for (uint32_t g = 0; g < N; ++g) {
        G.E[(g * 64 + j) * 2 + 0] = s_sp[g][j];
        G.E[(g * 64 + j) * 2 + 1] = s_t[g][j];
        G.walker[g * 64 + j] = s_w[g][j];
    }
    __syncthreads();  // s_mask complete (one wave: cheap)
    if (j + 1 < N) {
        const uint64_t mask = s_mask[j];
        G.swaplog[(size_t)(p % G.log_cap) * (N - 1) + j] = mask;
        G.acc[j] += (uint64_t)__popcll(mask);
        G.lastmask[j] = mask;
    }
    if (j == 0) G.lastmask[N - 1] = any ? 1ull : 0ull;

    // round trips 0 -> N-1 -> 0; this step ends at PT time p+1.  One slot
    // has no exchange partner and no pair of distinct end slots: its walkers
    // never move, and no round trip is counted.
    if (N < 2) return;
    const uint32_t now = p + 1;
    RoundTrip& r0 = G.rt[s_w[0][j] * 64 + j];
    if (r0.state == 2) {
        r0.count += 1;
        r0.sum += (uint64_t)(now - r0.t_last);
        r0.t_last = now;
        r0.state = 1;
    } else if (r0.state == 0) {
        r0.t_last = now;
        r0.state = 1;
    }
    RoundTrip& rtop = G.rt[s_w[N - 1][j] * 64 + j];
    if (rtop.state == 1) rtop.state = 2;
}

__global__ void __launch_bounds__(64)
k_pt(const GroupDev G, const uint32_t* __restrict__ ctr, uint32_t p_add) {
    pt_group(G, ctr[1] + p_add);
}

__global__ void __launch_bounds__(64)
k_pt_batched(const GroupDev* __restrict__ groups, const uint32_t* __restrict__ ctr, uint32_t p_add) {
    const GroupDev G = uniform_record(groups + blockIdx.x);
    pt_group(G, ctr[1] + p_add);
}

// Sweep and PT counters live on the device so that a captured graph can be
// replayed: every launch reads them and adds its own offset.
__global__ void k_advance(uint32_t* ctr, uint32_t dt, uint32_t dp) {
    if (threadIdx.x == 0) {
        ctr[0] += dt;
        ctr[1] += dp;
    }
}

// ---------------------------------------------------------------------------
// Apply the accepted exchanges of the latest PT step to the spins: at every
// site, the pairs' masked bit exchanges in ascending order (each word read
// and written once).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void swap_site(const GroupDev& G, uint32_t site) {
    const uint32_t N = G.N;
    uint64_t* S = G.spins + site;
    const size_t V = G.V;
    uint64_t cur = S[0];  // running content of slot g
    uint64_t orig = cur;  // what slot g held before this step
    for (uint32_t g = 0; g + 1 < N; ++g) {
        const uint64_t nx = S[(size_t)(g + 1) * V];
        const uint64_t d = (cur ^ nx) & G.lastmask[g];
        cur ^= d;
        if (cur != orig) S[(size_t)g * V] = cur;
        cur = nx ^ d;
        orig = nx;
    }
    if (cur != orig) S[(size_t)(N - 1) * V] = cur;
}

__global__ void __launch_bounds__(kSwapBlock) k_swap_apply(const GroupDev G) {
    if (G.N < 2 || G.lastmask[G.N - 1] == 0) return;
    const uint32_t site = blockIdx.x * kSwapBlock + threadIdx.x;
    if (site < G.V) swap_site(G, site);
}

__global__ void __launch_bounds__(kSwapBlock)
k_swap_apply_batched(const BatchPlan plan) {
    const BlockPlace at = locate<false>(plan, blockIdx.x);
    const GroupDev G = group_record<false>(plan, at.gi);
    if (G.N < 2 || G.lastmask[G.N - 1] == 0) return;
    const uint32_t site = at.local * kSwapBlock + threadIdx.x;
    if (site < G.V) swap_site(G, site);
}

// ---------------------------------------------------------------------------
// Initialisation.
// ---------------------------------------------------------------------------
// Couplings: lane j has J_{i,d} = -1 iff bit 0 of word 0 of Philox with
// counter (i, d, 3<<24, 0) under key j_seed[j] is set (i = x + L*y;
// d = 0: +x bond, d = 1: +y bond).
__global__ void k_init_couplings(const GroupDev G) {
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t P = G.L * G.L;
    if (b >= 2 * P) return;
    const uint32_t d = b / P, i = b - d * P;
    uint64_t w = 0;
    for (int j = 0; j < 64; ++j) {
        const uint64_t key = G.jseed[j];
        const uint4 o = philox(make_uint4(i, d, 3u << 24, 0u), (uint32_t)key, (uint32_t)(key >> 32));
        w |= (uint64_t)(o.x & 1u) << j;
    }
    (d == 0 ? G.Jx : G.Jy)[i] = w;
}

// Spins: word(s, g) = o0 | o1<<32 of Philox with counter (s, 0, 2<<24 | g, gid).
__global__ void k_init_spins(const GroupDev G) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t g = blockIdx.y;
    if (s >= G.V) return;
    const uint4 o = philox(make_uint4(s, 0u, (2u << 24) | g, G.gid), G.key0, G.key1);
    G.spins[(size_t)g * G.V + s] = lo_hi(o.x, o.y);
}

// Walkers at their own slots, trackers, counters and sums cleared; walker 0
// starts its clock at slot 0.
__global__ void k_init_state(const GroupDev G) {
    const uint32_t j = threadIdx.x;
    const uint32_t N = G.N;
    for (uint32_t g = 0; g < N; ++g) {
        G.walker[g * 64 + j] = g;
        RoundTrip r;
        r.state = (g == 0) ? 1u : 0u;
        r.t_last = 0;
        r.count = 0;
        r.pad = 0;
        r.sum = 0;
        G.rt[g * 64 + j] = r;
        for (int k = j; k < kCntStride; k += 64) G.cnt[g * kCntStride + k] = 0;
        for (int k = j; k < kSumStride; k += 64) G.sums[(size_t)g * kSumStride + k] = 0;
        for (int k = j; k < kHistBins; k += 64) G.hist[(size_t)g * kHistBins + k] = 0;
        G.E[(g * 64 + j) * 2 + 0] = 0;
        G.E[(g * 64 + j) * 2 + 1] = 0;
    }
    const uint32_t pairs = N > 1 ? N - 1 : 1;  // the acc region has max(N-1, 1) entries
    for (uint32_t g = j; g < N; g += 64) G.lastmask[g] = 0;
    for (uint32_t g = j; g < pairs; g += 64) G.acc[g] = 0;
    const size_t nlog = (size_t)G.log_cap * (N > 1 ? N - 1 : 1);
    for (size_t i = j; i < nlog; i += 64) G.swaplog[i] = 0;
}

__global__ void k_zero32(uint32_t* p, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ void k_philox(const uint32_t* in, uint32_t* out, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t* a = in + 6 * (size_t)i;
    const uint4 o = philox(make_uint4(a[0], a[1], a[2], a[3]), a[4], a[5]);
    uint32_t* b = out + 4 * (size_t)i;
    b[0] = o.x;
    b[1] = o.y;
    b[2] = o.z;
    b[3] = o.w;
}


// Random-number ceiling: thread i generates `blocks` Philox blocks with the
// counters the colour pass uses (a per-thread first word, block-uniform
// others: (i, 0, b, 0)) and stores the xor of all their output words.
__global__ void __launch_bounds__(256)
k_philox_probe(uint32_t* out, uint32_t n, uint32_t blocks, uint32_t k0, uint32_t k1) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t x = 0;
#pragma unroll 1
    for (uint32_t b = 0; b < blocks; ++b) {
        const uint4 o = philox(make_uint4(i, 0u, b, 0u), k0, k1);
        x ^= xor3(o.x, o.y, o.z) ^ o.w;
    }
    out[i] = x;
}

}  // namespace

// ------------------------------- launchers ---------------------------------

hipError_t launch_init_couplings(const GroupDev& g, hipStream_t s) {
    const uint32_t n = 2 * g.L * g.L;
    hipLaunchKernelGGL(k_init_couplings, dim3((n + 63) / 64), dim3(64), 0, s, g);
    return hipGetLastError();
}
hipError_t launch_init_spins(const GroupDev& g, hipStream_t s) {
    hipLaunchKernelGGL(k_init_spins, dim3((g.V + 255) / 256, g.N), dim3(256), 0, s, g);
    return hipGetLastError();
}
hipError_t launch_init_state(const GroupDev& g, hipStream_t s) {
    hipLaunchKernelGGL(k_init_state, dim3(1), dim3(64), 0, s, g);
    return hipGetLastError();
}
hipError_t launch_half_sweep(const GroupDev& g, uint32_t colour, const uint32_t* ctr,
                             uint32_t t_add, hipStream_t s) {
    hipLaunchKernelGGL(k_half_sweep, dim3(sweep_blocks_per_slot(g.V, g.tile), g.N), dim3(kSweepBlock), 0, s,
                       g, colour, ctr, t_add);
    return hipGetLastError();
}
hipError_t launch_energy(const GroupDev& g, int32_t* cnt, hipStream_t s) {
    const uint32_t planes = tile_for(g.Ltau, kEnergyPlanesSlot);
    hipLaunchKernelGGL(k_energy, dim3(energy_blocks_per_slot(g.V, planes), g.N),
                       dim3(kEnergyBlock), 0, s, g, cnt, planes);
    return hipGetLastError();
}
hipError_t launch_pt(const GroupDev& g, const uint32_t* ctr, uint32_t p_add, hipStream_t s) {
    hipLaunchKernelGGL(k_pt, dim3(1), dim3(64), 0, s, g, ctr, p_add);
    return hipGetLastError();
}
hipError_t launch_swap_apply(const GroupDev& g, hipStream_t s) {
    hipLaunchKernelGGL(k_swap_apply, dim3(swap_blocks(g.V)), dim3(kSwapBlock), 0, s, g);
    return hipGetLastError();
}
hipError_t launch_zero32(void* p, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       (uint32_t*)p, n);
    return hipGetLastError();
}
hipError_t launch_philox(const uint32_t* in, uint32_t* out, uint32_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_philox, dim3((n + 63) / 64), dim3(64), 0, s, in, out, n);
    return hipGetLastError();
}
hipError_t launch_philox_probe(uint32_t* out, uint32_t n, uint32_t blocks, uint64_t key,
                              hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_philox_probe, dim3((n + 255) / 256), dim3(256), 0, s, out, n, blocks,
                       (uint32_t)key, (uint32_t)(key >> 32));
    return hipGetLastError();
}
hipError_t launch_half_sweep_batched(const BatchPlan& plan, uint32_t colour, const uint32_t* ctr,
                                     uint32_t t_add, hipStream_t s) {
    if (plan.n_blocks == 0) return hipSuccess;
    if (plan.same_shape)
        hipLaunchKernelGGL(k_half_sweep_batched<true>, dim3(plan.n_blocks), dim3(kSweepBlock), 0, s,
                           plan, colour, ctr, t_add);
    else
        hipLaunchKernelGGL(k_half_sweep_batched<false>, dim3(plan.n_blocks), dim3(kSweepBlock), 0,
                           s, plan, colour, ctr, t_add);
    return hipGetLastError();
}
hipError_t launch_chunk_fused(const BatchPlan& slots, const uint32_t* ctr, uint32_t n_sweeps,
                              uint32_t lds_words, hipStream_t s) {
    if (slots.n_blocks == 0) return hipSuccess;
    const size_t lds = (size_t)lds_words * sizeof(uint64_t);
    if (lds > 48 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)k_chunk_fused,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_chunk_fused, dim3(slots.n_blocks), dim3(kSweepBlock), lds, s, slots, ctr,
                       n_sweeps, lds_words);
    return hipGetLastError();
}

hipError_t launch_energy_batched(const BatchPlan& plan, hipStream_t s) {
    if (plan.n_blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_energy_batched, dim3(plan.n_blocks), dim3(kEnergyBlock), 0, s, plan);
    return hipGetLastError();
}
hipError_t launch_pt_batched(const GroupDev* groups, uint32_t n_groups, const uint32_t* ctr,
                             uint32_t p_add, hipStream_t s) {
    if (n_groups == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pt_batched, dim3(n_groups), dim3(64), 0, s, groups, ctr, p_add);
    return hipGetLastError();
}
hipError_t launch_advance(uint32_t* ctr, uint32_t dt, uint32_t dp, hipStream_t s) {
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, ctr, dt, dp);
    return hipGetLastError();
}
hipError_t launch_swap_apply_batched(const BatchPlan& plan, hipStream_t s) {
    if (plan.n_blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_swap_apply_batched, dim3(plan.n_blocks), dim3(kSwapBlock), 0, s, plan);
    return hipGetLastError();
}

}  // namespace qsg
