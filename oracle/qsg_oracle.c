/*
 * Plain CPU oracle for the MCQSG Metropolis + parallel-tempering sweep.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product links, loads or calls
 * this file; only the tests, the smoke check and the CPU baseline of the
 * benchmark do.  It shares no code, header or table generator with the HIP
 * path.  It updates one spin (one bit of one lane at one site in one slot)
 * at a time, in the most direct form the definitions allow.
 *
 * Model (paper: Sec. 1, Eqs. (1)-(3), Trotter-Suzuki map to an
 * L x L x L_tau prism; Sec. 2.1, checkerboard Metropolis and parallel
 * tempering).  Two ladders.  Transverse-field ladder (two-coupling form):
 * spatial bonds carry k*J with k = beta/L_tau, temporal bonds carry
 * kp_g = -1/2 ln tanh(beta*Gamma_g/L_tau), and PT exchanges Gamma values with
 * the time-bond energy.  Coupling ladder (the paper's own form): one
 * coupling k_g on every bond of slot g, PT exchanges k values with the whole
 * energy.  The tables (built by the caller) carry the couplings; the chain
 * only needs to know which energy the exchange uses.
 *
 * Conventions (readings of the paper, listed in the design notes):
 *  - spins: uint64 word per (slot g, tau, y, x); bit j = lane j; bit 1 <=> S = -1
 *    (bit convention of App. D);
 *  - couplings: Jx[y][x] on bond (x,y)-(x+1,y), Jy[y][x] on (x,y)-(x,y+1);
 *    bit 1 <=> J = -1; bonds form a multiset indexed by (site, direction);
 *  - colour of (x,y,tau) is (x+y+tau) mod 2; red (0) is updated first;
 *  - acceptance: r_j <= thr[g][n_s][n_t], thr = ceil(2^32 * min(1, e^-dE)) - 1,
 *    tables supplied by the caller (built with mpmath);
 *  - random numbers: Philox4x32-10 (Salmon et al., SC'11; the generator the
 *    paper uses in Sec. 2.1.1), counters tied to the lattice update so the
 *    trajectory does not depend on work distribution (Sec. 2.1.1 footnote).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------------------
 * Philox4x32-10 from its published definition: ten rounds of
 *   (hi0,lo0) = M0*c0, (hi1,lo1) = M1*c2,
 *   c' = (hi1^c1^k0, lo1, hi0^c3^k1, lo0),
 * with the Weyl key increments applied between rounds.
 * ------------------------------------------------------------------------- */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                          uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void philox_u64seed(uint32_t a, uint32_t b, uint32_t c, uint32_t d,
                           uint64_t seed, uint32_t out[4]) {
    uint32_t ctr[4] = {a, b, c, d};
    uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
    oracle_philox4x32_10(ctr, key, out);
}

/* Metropolis random numbers of the 64 lanes at (site s, sweep t, slot g).
 * Domain 0: block q (0..15) has counter (s, t, (g<<4)|q, group_id).  Block q
 * yields level 2q = o0 | o1<<32 and level 2q+1 = o2 | o3<<32; lane j's
 * 32-bit number has bit (31-b) equal to bit j of level b. */
void oracle_metropolis_r(uint64_t seed, uint32_t group_id, uint32_t s,
                         uint32_t t, uint32_t g, uint32_t r[64]) {
    uint64_t level[32];
    for (uint32_t q = 0; q < 16; ++q) {
        uint32_t o[4];
        philox_u64seed(s, t, (0u << 24) | (g << 4) | q, group_id, seed, o);
        level[2 * q] = (uint64_t)o[0] | ((uint64_t)o[1] << 32);
        level[2 * q + 1] = (uint64_t)o[2] | ((uint64_t)o[3] << 32);
    }
    for (int j = 0; j < 64; ++j) {
        uint32_t v = 0;
        for (int b = 0; b < 32; ++b)
            v |= (uint32_t)((level[b] >> j) & 1u) << (31 - b);
        r[j] = v;
    }
}

/* PT random number of lane j at PT step p for pair (g, g+1).
 * Domain 1: counter (j>>2, p, (1<<24)|g, group_id), output word j&3. */
uint32_t oracle_pt_r(uint64_t seed, uint32_t group_id, uint32_t p, uint32_t g,
                     uint32_t j) {
    uint32_t o[4];
    philox_u64seed(j >> 2, p, (1u << 24) | g, group_id, seed, o);
    return o[j & 3];
}

static inline int bit_of(uint64_t w, int j) { return (int)((w >> j) & 1u); }

/* Couplings: lane j has J_{i,d} = -1 iff bit 0 of o0 of Philox with counter
 * (i = x + L*y, d, 3<<24, 0) under key j_seed[j] is set.  d=0: +x bond,
 * d=1: +y bond.  Output words: Jx[i], Jy[i], bit j = lane j. */
void oracle_init_couplings(int L, const uint64_t j_seed[64], uint64_t *Jx,
                           uint64_t *Jy) {
    for (int i = 0; i < L * L; ++i) {
        uint64_t wx = 0, wy = 0;
        for (int j = 0; j < 64; ++j) {
            uint32_t o[4];
            philox_u64seed((uint32_t)i, 0u, 3u << 24, 0u, j_seed[j], o);
            wx |= (uint64_t)(o[0] & 1u) << j;
            philox_u64seed((uint32_t)i, 1u, 3u << 24, 0u, j_seed[j], o);
            wy |= (uint64_t)(o[0] & 1u) << j;
        }
        Jx[i] = wx;
        Jy[i] = wy;
    }
}

/* Initial spins: word(s, g) = o0 | o1<<32 of Philox with counter
 * (s, 0, (2<<24)|g, group_id), s = x + L*(y + L*tau). */
void oracle_init_spins(int L, int Ltau, int N, uint32_t group_id, uint64_t seed,
                       uint32_t slot_base, uint64_t *spins) {
    size_t V = (size_t)L * L * Ltau;
    for (int g = 0; g < N; ++g)
        for (size_t s = 0; s < V; ++s) {
            uint32_t o[4];
            philox_u64seed((uint32_t)s, 0u, (2u << 24) | ((uint32_t)g + slot_base),
                           group_id, seed, o);
            spins[(size_t)g * V + s] = (uint64_t)o[0] | ((uint64_t)o[1] << 32);
        }
}

/* -------------------------- lattice helpers ------------------------------ */
typedef struct {
    int L, Ltau;
    int anti; /* 1: antiperiodic along tau, S(tau + L_tau) = -S(tau) (Sec. 1) */
} lat_t;

/* Sign of the time bond from slice tau to tau+1: -1 on the bond that wraps
 * round an antiperiodic prism. */
static inline int tbond_sign(const lat_t *a, int tau) {
    return (a->anti && tau == a->Ltau - 1) ? -1 : +1;
}

static inline size_t site(const lat_t *a, int x, int y, int tau) {
    return (size_t)x + (size_t)a->L * ((size_t)y + (size_t)a->L * (size_t)tau);
}
/* periodic neighbour coordinate; v is in [-1, n] */
static inline int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

/* Spin value (+1/-1) of lane j at a site of one slot. */
static inline int spin_val(const uint64_t *S, size_t idx, int j) {
    return bit_of(S[idx], j) ? -1 : +1;
}
static inline int coup_val(const uint64_t *J, int i, int j) {
    return bit_of(J[i], j) ? -1 : +1;
}

/* The seven spin words and four coupling words around a site. */
typedef struct {
    uint64_t c, xp, xm, yp, ym, tp, tm; /* centre and its six neighbours   */
    uint64_t jxp, jxm, jyp, jym;        /* couplings of the four space bonds */
    int stp, stm;                       /* signs of the +tau and -tau bonds  */
} nbhd_t;

static void load_nbhd(const lat_t *a, const uint64_t *S, const uint64_t *Jx,
                      const uint64_t *Jy, int x, int y, int tau, nbhd_t *n) {
    int L = a->L;
    int xp = wrap(x + 1, L), xm = wrap(x - 1, L);
    int yp = wrap(y + 1, L), ym = wrap(y - 1, L);
    int tp = wrap(tau + 1, a->Ltau), tm = wrap(tau - 1, a->Ltau);
    n->c = S[site(a, x, y, tau)];
    n->xp = S[site(a, xp, y, tau)];
    n->xm = S[site(a, xm, y, tau)];
    n->yp = S[site(a, x, yp, tau)];
    n->ym = S[site(a, x, ym, tau)];
    n->tp = S[site(a, x, y, tp)];
    n->tm = S[site(a, x, y, tm)];
    /* bond to +x carries Jx at (x,y); the bond to -x is the +x bond of (x-1,y) */
    n->jxp = Jx[x + L * y];
    n->jxm = Jx[xm + L * y];
    n->jyp = Jy[x + L * y];
    n->jym = Jy[x + L * ym];
    n->stp = tbond_sign(a, tau);
    n->stm = tbond_sign(a, tm);
}

static inline int pm(uint64_t w, int j) { return bit_of(w, j) ? -1 : +1; }

/* Number of unsatisfied spatial bonds (of 4) and temporal bonds (of 2)
 * around lane j's spin; a bond with J*S*S' < 0 is unsatisfied (J = the
 * bond's sign for time bonds). */
static void lane_classes(const nbhd_t *n, int j, int *ns, int *nt) {
    int s0 = pm(n->c, j);
    int u = 0;
    if (pm(n->jxp, j) * s0 * pm(n->xp, j) < 0) u++;
    if (pm(n->jxm, j) * s0 * pm(n->xm, j) < 0) u++;
    if (pm(n->jyp, j) * s0 * pm(n->yp, j) < 0) u++;
    if (pm(n->jym, j) * s0 * pm(n->ym, j) < 0) u++;
    int v = 0;
    if (n->stp * s0 * pm(n->tp, j) < 0) v++;
    if (n->stm * s0 * pm(n->tm, j) < 0) v++;
    *ns = u;
    *nt = v;
}

/* Exported for the exact tests: (n_s, n_t) of lane 0 at every site for a
 * batch of single-lane configurations.  cfg[b*V + s] holds the spin word of
 * site s in configuration b. */
void oracle_site_classes(int L, int Ltau, int anti, const uint64_t *Jx, const uint64_t *Jy,
                         const uint64_t *cfg, int64_t n_cfg, int lane,
                         uint8_t *ns_out, uint8_t *nt_out) {
    lat_t a = {L, Ltau, anti};
    size_t V = (size_t)L * L * Ltau;
    for (int64_t b = 0; b < n_cfg; ++b) {
        const uint64_t *S = cfg + (size_t)b * V;
        for (int tau = 0; tau < Ltau; ++tau)
            for (int y = 0; y < L; ++y)
                for (int x = 0; x < L; ++x) {
                    int ns, nt;
                    nbhd_t n;
                    load_nbhd(&a, S, Jx, Jy, x, y, tau, &n);
                    lane_classes(&n, lane, &ns, &nt);
                    size_t s = site(&a, x, y, tau);
                    ns_out[(size_t)b * V + s] = (uint8_t)ns;
                    nt_out[(size_t)b * V + s] = (uint8_t)nt;
                }
    }
}

/* From-scratch bond sums per lane for one slot (Eq. (3) split into its
 * spatial and temporal parts):
 *   Bsp = sum over sites of Jx S S_{+x} + Jy S S_{+y},
 *   Bt  = sum over sites of S_tau S_{tau+1}, with S_{L_tau} = -S_0 when
 *         antiperiodic. */
static void recompute_B(const lat_t *a, const uint64_t *S, const uint64_t *Jx,
                        const uint64_t *Jy, int64_t Bsp[64], int64_t Bt[64]) {
    int L = a->L;
    for (int j = 0; j < 64; ++j) {
        int64_t bs = 0, bt = 0;
        for (int tau = 0; tau < a->Ltau; ++tau)
            for (int y = 0; y < L; ++y)
                for (int x = 0; x < L; ++x) {
                    int s0 = spin_val(S, site(a, x, y, tau), j);
                    bs += coup_val(Jx, x + L * y, j) * s0 *
                          spin_val(S, site(a, wrap(x + 1, L), y, tau), j);
                    bs += coup_val(Jy, x + L * y, j) * s0 *
                          spin_val(S, site(a, x, wrap(y + 1, L), tau), j);
                    bt += tbond_sign(a, tau) * s0 *
                          spin_val(S, site(a, x, y, wrap(tau + 1, a->Ltau)), j);
                }
        Bsp[j] = bs;
        Bt[j] = bt;
    }
}

/* Same-time, same-tau overlap of lane pairs (2p, 2p+1): sum over sites of
 * S^{2p} S^{2p+1} (the Q of App. E with tau1 = tau2 and t1 = t2). */
static void overlap_pairs(const lat_t *a, const uint64_t *S, int64_t q[32]) {
    size_t V = (size_t)a->L * a->L * a->Ltau;
    for (int p = 0; p < 32; ++p) {
        int64_t acc = 0;
        for (size_t s = 0; s < V; ++s)
            acc += spin_val(S, s, 2 * p) * spin_val(S, s, 2 * p + 1);
        q[p] = acc;
    }
}

void oracle_recompute(int L, int Ltau, int anti, int N, const uint64_t *Jx,
                      const uint64_t *Jy, const uint64_t *spins, int32_t *Bsp,
                      int32_t *Bt, int64_t *q) {
    lat_t a = {L, Ltau, anti};
    size_t V = (size_t)L * L * Ltau;
    for (int g = 0; g < N; ++g) {
        int64_t bs[64], bt[64], qq[32];
        recompute_B(&a, spins + (size_t)g * V, Jx, Jy, bs, bt);
        overlap_pairs(&a, spins + (size_t)g * V, qq);
        for (int j = 0; j < 64; ++j) {
            Bsp[g * 64 + j] = (int32_t)bs[j];
            Bt[g * 64 + j] = (int32_t)bt[j];
        }
        for (int p = 0; p < 32; ++p) q[g * 32 + p] = qq[p];
    }
}

/* ---------------------------- the chain ---------------------------------- */
typedef struct {
    int32_t L, Ltau, N;
    uint32_t group_id;
    uint64_t mc_seed;
    const uint32_t *thr;     /* [N][5][3]: index (g*5 + ns)*3 + nt          */
    const uint8_t *pt_equal; /* [N-1]: 1 if kp_g == kp_{g+1} exactly      */
    const uint32_t *sw_len;  /* [N-1]: number of positive table entries  */
    const uint64_t *sw_off;  /* [N-1]: offset of pair g's entries        */
    const uint32_t *sw_thr;  /* entry m-1 of pair g: threshold for D=-4m */
    const uint64_t *Jx, *Jy; /* [L*L] each                               */
    uint64_t *spins;         /* [N][Ltau][L][L]                          */
    /* state, all [N][64] unless noted */
    int32_t *Bsp, *Bt;       /* tracked bond sums (in/out)               */
    uint8_t *walker;         /* walker label at (slot, lane)             */
    uint8_t *rt_state;       /* per (walker, lane): 0 unstarted, 1 up, 2 down */
    uint32_t *rt_tlast;      /* PT time of the last visit to slot 0      */
    uint32_t *rt_count;      /* completed round trips                    */
    uint64_t *rt_sum;        /* sum of round-trip durations (PT steps)   */
    uint64_t *acc;           /* [N-1] accepted swaps, all lanes          */
    uint64_t *swaplog;       /* [log_cap][N-1], row p % log_cap          */
    uint64_t log_cap;
    int64_t *sum_Bsp, *sum_Bt; /* [N][64] sums of pre-swap values per PT step */
    int64_t *sum_q, *sum_q2;   /* [N][32]                                   */
    uint64_t *counters;      /* [0] sweeps done t, [1] PT steps done p   */
    uint32_t *hist;          /* [N][1024] histogram of u = (V - Bt)/2 at every PT
                                step before the exchanges, bin = u*1024/(V+1) */
    uint32_t slot_base;      /* slot g of this state is slot g+slot_base of the
                                full ladder (random-number counters only); lets a
                                test follow a few slots of a large group between
                                PT steps, where slots evolve independently     */
    uint32_t tau_anti;       /* 1: antiperiodic boundary along tau        */
    uint32_t exch_all;       /* 0: the slots differ in the time coupling only
                                (transverse-field ladder), the exchange uses Bt;
                                1: one coupling k_g on every bond (k ladder), the
                                exchange uses the whole energy Bsp + Bt        */
} oracle_state;

static void pt_step(oracle_state *st, int *failed) {
    lat_t a = {st->L, st->Ltau, (int)st->tau_anti};
    const int N = st->N;
    const size_t V = (size_t)st->L * st->L * st->Ltau;
    const uint32_t p = (uint32_t)st->counters[1];

    /* The measurement of App. A: tracked sums must equal sums recomputed
     * from the configuration, and the recomputed values enter the per-step
     * sums and histograms -- for every group, one slot included (the energy
     * measurement does not depend on the exchange).  Slots are
     * independent here, so OpenMP may split them. */
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
    for (int g = 0; g < N; ++g) {
        int64_t bs[64], bt[64], qq[32];
        recompute_B(&a, st->spins + (size_t)g * V, st->Jx, st->Jy, bs, bt);
        overlap_pairs(&a, st->spins + (size_t)g * V, qq);
        for (int j = 0; j < 64; ++j) {
            if (bs[j] != st->Bsp[g * 64 + j] || bt[j] != st->Bt[g * 64 + j])
                bad = 1;
            st->sum_Bsp[g * 64 + j] += bs[j];
            st->sum_Bt[g * 64 + j] += bt[j];
            /* bt = V - 2u with u the number of unsatisfied time bonds */
            int64_t u = ((int64_t)V - bt[j]) / 2;
            st->hist[(size_t)g * 1024 + (size_t)(u * 1024 / ((int64_t)V + 1))] += 1;
        }
        for (int q = 0; q < 32; ++q) {
            st->sum_q[g * 32 + q] += qq[q];
            st->sum_q2[g * 32 + q] += qq[q] * qq[q];
        }
    }
    if (bad) *failed = 1;

    if (N < 2) {
        /* one slot: no exchange partner and no pair of distinct end slots,
         * so there is no exchange and no round trip */
        st->counters[1] = p + 1;
        return;
    }

    /* Pairs in ascending order; each decision sees the state left by the
     * previous one.  Swap probability min(1, e^{(c_g - c_{g+1}) D}) (Sec. 2.1,
     * the exchange probability): for a transverse-field ladder c = kp, the
     * coupling that differs between slots, and D = Bt[g+1] - Bt[g]; for a k
     * ladder c = k and D is the change of the whole exponent Bsp + Bt
     * (Eq. (3)). */
    for (int g = 0; g + 1 < N; ++g) {
        uint64_t mask = 0;
        for (int j = 0; j < 64; ++j) {
            int64_t D = (int64_t)st->Bt[(g + 1) * 64 + j] - st->Bt[g * 64 + j];
            if (st->exch_all)
                D += (int64_t)st->Bsp[(g + 1) * 64 + j] - st->Bsp[g * 64 + j];
            int accept;
            if (st->pt_equal[g] || D >= 0) {
                accept = 1;
            } else {
                uint64_t m = (uint64_t)(-D) / 4u;
                uint32_t thr = (m >= 1 && m <= st->sw_len[g])
                                   ? st->sw_thr[st->sw_off[g] + (m - 1)]
                                   : 0u;
                uint32_t r = oracle_pt_r(st->mc_seed, st->group_id, p,
                                         (uint32_t)g, (uint32_t)j);
                accept = (r <= thr);
            }
            if (accept) {
                mask |= 1ull << j;
                int32_t t;
                t = st->Bsp[g * 64 + j];
                st->Bsp[g * 64 + j] = st->Bsp[(g + 1) * 64 + j];
                st->Bsp[(g + 1) * 64 + j] = t;
                t = st->Bt[g * 64 + j];
                st->Bt[g * 64 + j] = st->Bt[(g + 1) * 64 + j];
                st->Bt[(g + 1) * 64 + j] = t;
                uint8_t w = st->walker[g * 64 + j];
                st->walker[g * 64 + j] = st->walker[(g + 1) * 64 + j];
                st->walker[(g + 1) * 64 + j] = w;
            }
        }
        /* move lane j's configuration between the two slots, bit by bit */
        uint64_t *A = st->spins + (size_t)g * V;
        uint64_t *B = st->spins + (size_t)(g + 1) * V;
        for (size_t s = 0; s < V; ++s)
            for (int j = 0; j < 64; ++j)
                if ((mask >> j) & 1u) {
                    uint64_t ba = (A[s] >> j) & 1u, bb = (B[s] >> j) & 1u;
                    A[s] = (A[s] & ~(1ull << j)) | (bb << j);
                    B[s] = (B[s] & ~(1ull << j)) | (ba << j);
                }
        st->swaplog[(p % st->log_cap) * (uint64_t)(N - 1) + g] = mask;
        st->acc[g] += (uint64_t)__builtin_popcountll(mask);
    }

    /* Round trips: slot 0 -> slot N-1 -> slot 0, clock started at the first
     * visit to slot 0; times in PT steps (this step ends at time p+1). */
    uint32_t now = p + 1;
    for (int j = 0; j < 64; ++j) {
        int w0 = st->walker[0 * 64 + j];
        size_t i0 = (size_t)w0 * 64 + j;
        if (st->rt_state[i0] == 2) {
            st->rt_count[i0] += 1;
            st->rt_sum[i0] += (uint64_t)(now - st->rt_tlast[i0]);
            st->rt_tlast[i0] = now;
            st->rt_state[i0] = 1;
        } else if (st->rt_state[i0] == 0) {
            st->rt_tlast[i0] = now;
            st->rt_state[i0] = 1;
        }
        int wt = st->walker[(N - 1) * 64 + j];
        size_t it = (size_t)wt * 64 + j;
        if (st->rt_state[it] == 1) st->rt_state[it] = 2;
    }
    st->counters[1] = p + 1;
}

/* One colour pass over one slot. */
static void colour_pass(oracle_state *st, int g, int colour, uint32_t t) {
    lat_t a = {st->L, st->Ltau, (int)st->tau_anti};
    const size_t V = (size_t)st->L * st->L * st->Ltau;
    uint64_t *S = st->spins + (size_t)g * V;
    const uint32_t *thr = st->thr + (size_t)g * 15;
    for (int tau = 0; tau < st->Ltau; ++tau)
        for (int y = 0; y < st->L; ++y)
            for (int x = 0; x < st->L; ++x) {
                if (((x + y + tau) & 1) != colour) continue;
                size_t s = site(&a, x, y, tau);
                uint32_t r[64];
                oracle_metropolis_r(st->mc_seed, st->group_id, (uint32_t)s, t,
                                    (uint32_t)g + st->slot_base, r);
                /* Neighbours have the other colour, and flipping lane j
                 * only touches bit j of the centre, so one read serves all
                 * 64 lanes. */
                nbhd_t n;
                load_nbhd(&a, S, st->Jx, st->Jy, x, y, tau, &n);
                for (int j = 0; j < 64; ++j) {
                    int ns, nt;
                    lane_classes(&n, j, &ns, &nt);
                    if (r[j] <= thr[ns * 3 + nt]) {
                        S[s] ^= 1ull << j;
                        st->Bsp[g * 64 + j] += 4 * ns - 8;
                        st->Bt[g * 64 + j] += 4 * nt - 4;
                    }
                }
            }
}

/* Run n_sweeps full sweeps (red pass then blue pass over every slot) and a
 * PT step after every sweep t with (t+1) % pt_every == 0 (pt_every = 0: no
 * PT).  Returns 0, or 1 if tracked and recomputed bond sums ever differed. */
int oracle_run(oracle_state *st, uint64_t n_sweeps, uint32_t pt_every,
               int nthreads) {
    int failed = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    for (uint64_t it = 0; it < n_sweeps; ++it) {
        uint32_t t = (uint32_t)st->counters[0];
        for (int colour = 0; colour < 2; ++colour) {
            /* slots do not interact inside a colour pass */
#pragma omp parallel for schedule(dynamic, 1)
            for (int g = 0; g < st->N; ++g) colour_pass(st, g, colour, t);
        }
        st->counters[0] = (uint64_t)t + 1;
        if (pt_every && ((uint64_t)t + 1) % pt_every == 0) pt_step(st, &failed);
    }
    return failed;
}

/* One PT step on demand (outside the sweep cadence). */
int oracle_pt_step(oracle_state *st) {
    int failed = 0;
    pt_step(st, &failed);
    return failed;
}

size_t oracle_state_size(void) { return sizeof(oracle_state); }
