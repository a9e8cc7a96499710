/*
 * qsg.h -- C ABI of the MI355X MCQSG hot path: Metropolis plus parallel
 * tempering over the Trotter-Suzuki (2+1)-D lattice of the 2D +-J quantum
 * Ising spin glass (paper: "The QISG suite", Sec. 1 Eqs. (1)-(3), Sec. 2.1).
 *
 * Model.  Spins S(x,y,tau) = +-1 on an L x L x L_tau prism, periodic in
 * space and periodic or antiperiodic in tau (Sec. 1; see tau_boundary).
 * Space bonds (x,y)-(x+1,y) and (x,y)-(x,y+1) carry J = +-1 and coupling
 * k = beta/L_tau; time bonds (x,y,tau)-(x,y,tau+1) carry
 * kp_g = -1/2 ln tanh(beta Gamma_g / L_tau) (two-coupling form; the paper's
 * equal-coupling form, Sec. 1, is kp = k: see ladder_kind).  A configuration
 * at slot g has weight exp(k Bsp + kp_g Bt), with Bsp the sum of J S S' over
 * space bonds and Bt the sum of S S' over time bonds (Eq. (3) split in two).
 *
 * Packing.  A *group* is 64 independent bit-lanes that share L, L_tau,
 * beta, the Gamma ladder and the Monte Carlo key.  Lane j of every word is
 * one chain ("replica"); lanes may share one disorder sample or each carry
 * their own (per-lane coupling seeds).  Spins of a group are uint64 words
 * laid out [slot g][tau][y][x]; bit j is lane j; bit 1 <=> S = -1 (the bit
 * convention of App. D).  Couplings are uint64 words Jx[y][x], Jy[y][x],
 * bit 1 <=> J = -1.  Slot g always holds Gamma_g (ascending ladder).
 *
 * Update.  One sweep = red pass then blue pass, colour (x+y+tau) mod 2,
 * red = 0 (checkerboard, Sec. 2.1).  A spin with n_s unsatisfied space bonds
 * and n_t unsatisfied time bonds is flipped iff r <= thr[g][n_s][n_t] with
 * thr = ceil(2^32 min(1, e^{-dE})) - 1 and dE = 4k(2-n_s) + 4kp_g(1-n_t);
 * r is lane j's 32-bit Philox4x32-10 number (Sec. 2.1.1) for counter
 * (site, sweep, g<<4 | q, group_id): block q gives bit-levels 2q and 2q+1,
 * bit (31-b) of r is bit j of level b.  After every `pt_every`-th sweep a
 * parallel-tempering step (Sec. 2.1, exchange probability
 * min(1, e^{(kp_g - kp_{g+1}) (Bt[g+1]-Bt[g])})) visits pairs g = 0..N-2 in
 * order, each lane independently, and moves accepted lanes' configurations
 * between the two slots.  All decisions are integer comparisons, so results
 * are bit-exact and do not depend on launch configuration.
 *
 * Conventions.
 *  - Memory: the caller owns every device buffer.  qsg_create carves its
 *    state out of one caller-allocated device workspace of
 *    qsg_workspace_bytes() bytes, which must stay alive until qsg_destroy.
 *    The library allocates no device memory (hipGraph objects aside).
 *    Host buffers passed in are read before the call returns.
 *  - Streams: work is enqueued on the caller's HIP stream.  qsg_measure,
 *    qsg_get_* and qsg_sync synchronise that stream.
 *  - Errors: functions return QSG_OK or a negative qsg_status and never
 *    abort or throw.  Invalid arguments leave the context unchanged
 *    (QSG_E_INVALID); qsg_last_error() describes the last failure.  A device
 *    error marks the context failed; later calls return QSG_E_STATE.
 *  - Threads: one context must not be used from two threads at once.
 */
#ifndef QSG_H
#define QSG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qsg_ctx qsg_ctx;
typedef int32_t qsg_status;

#define QSG_OK 0
#define QSG_E_INVALID (-1)     /* bad argument; nothing changed          */
#define QSG_E_UNSUPPORTED (-2) /* valid but outside what is built        */
#define QSG_E_DEVICE (-3)      /* a HIP call failed                      */
#define QSG_E_STATE (-4)       /* context failed earlier / wrong state   */
#define QSG_E_BUFFER (-5)      /* caller buffer too small                */
#define QSG_E_INTERRUPTED (-6) /* deadline reached between chunks        */

#define QSG_MAX_GAMMA 64

/* Description of one group (64 lanes). */
typedef struct {
    uint32_t L;              /* linear size, even, 2..256                     */
    uint32_t L_tau;          /* imaginary-time slices, even, 2..65536         */
    double beta;             /* inverse temperature, > 0; k = beta / L_tau    */
    uint32_t n_gamma;        /* ladder points (slots), 1..64                  */
    uint32_t group_id;       /* Philox counter word 3 of this group           */
    uint64_t mc_seed;        /* Philox key (lo, hi) of spins, sweeps and PT   */
    uint64_t j_seed[64];     /* Philox key of lane j's couplings              */
    uint32_t swap_table_cap; /* max swap-table entries per pair (0 = 4096)    */
    uint32_t ladder_kind;    /* QSG_LADDER_GAMMA (0) or QSG_LADDER_K (1)      */
    uint32_t tau_boundary;   /* QSG_TAU_PERIODIC (0) or QSG_TAU_ANTIPERIODIC (1) */
    uint32_t reserved;       /* must be 0                                     */
} qsg_group_desc;

/* Boundary along imaginary time (Sec. 1 allows both): periodic,
 * S(tau + L_tau) = S(tau), or antiperiodic, S(tau + L_tau) = -S(tau): the
 * time bond from slice L_tau-1 to slice 0 then counts with the opposite
 * sign in Bt and in the Metropolis classes. */
#define QSG_TAU_PERIODIC 0u
#define QSG_TAU_ANTIPERIODIC 1u

/* Ladder kinds.  GAMMA: slot g runs the two-coupling form at transverse
 * field Gamma_g (k = beta/L_tau on space bonds, kp_g on time bonds) and PT
 * exchanges Gamma values with the time-bond energy (qsg_set_gamma_ladder).
 * K: the paper's own parametrisation (Sec. 1, Eqs. (2)-(3); k list of
 * App. C): slot g has one coupling k_g on every bond (the transverse field
 * is -ln tanh(k_g)/(2 k_g)), PT exchanges k values with the full energy,
 * probability min(1, e^{(k_g - k_{g+1})(B[g+1]-B[g])}), B = Bsp + Bt
 * (Sec. 2.1); set with qsg_set_k_ladder.  beta is unused (still > 0). */
#define QSG_LADDER_GAMMA 0u
#define QSG_LADDER_K 1u

/* Run-wide settings. */
typedef struct {
    uint32_t pt_every;    /* PT step after sweep t if (t+1) % pt_every == 0; 0 = none */
    uint32_t swaplog_cap; /* PT steps kept in the swap log ring (>= 1)        */
    uint32_t sweep_split; /* schedule of the colour pass: Philox blocks every
                             word goes through before the words still undecided
                             are packed into fewer waves (1..16; 16 = never;
                             0 = default 4).  Results do not depend on it.     */
    uint32_t tau_tile;    /* schedule of the colour pass: tau planes a thread
                             walks along one column (it updates tau_tile/2 words;
                             0 = default 8).  Each group uses the largest power
                             of two <= tau_tile (2..32) dividing its L_tau.
                             Results do not depend on it.                      */
} qsg_run_config;

/* qsg_sweep flags */
#define QSG_PLAIN 0u    /* one launch per group and pass (per-sample launches) */
#define QSG_BATCHED 1u  /* one launch per pass over every group                */
#define QSG_GRAPH 2u    /* with QSG_BATCHED: replay a captured HIP graph       */
#define QSG_NO_PT 4u    /* skip the PT steps that fall due                     */
#define QSG_FUSED 8u    /* with QSG_BATCHED: the sweeps of a whole PT chunk in
                           one launch, one block per slot (small slots from LDS);
                           pays off only when every slot is small (one block
                           then replaces a launch per colour pass); a slot of
                           many blocks' worth of words runs serially in its one
                           block, far slower than the per-pass form          */

/* qsg_measure selectors (one at a time) */
#define QSG_M_ENERGY 1u    /* int32 [G][N][64][2]: (Bsp, Bt) recomputed now      */
#define QSG_M_OVERLAP 2u   /* int64 [G][N][32]: sum_sites S^{2p} S^{2p+1}, now   */
#define QSG_M_ACCEPT 3u    /* uint64 [G][N-1]: accepted exchanges, all lanes     */
#define QSG_M_WALKERS 4u   /* uint8  [G][N][64]: walker label at (slot, lane)    */
#define QSG_M_SWAPLOG 5u   /* uint64 [G][cap][N-1]: masks, row p % cap           */
#define QSG_M_ROUNDTRIP 6u /* qsg_roundtrip [G][N][64] by (walker, lane)         */
#define QSG_M_SUMS 7u      /* int64 [G][N][192]: per PT step sums of pre-exchange
                              Bsp[64], Bt[64], q[32], q^2[32]                   */
#define QSG_M_COUNTERS 8u  /* uint64 [2]: sweeps done, PT steps done            */
#define QSG_M_HIST 9u      /* uint32 [G][N][1024]: per PT step and lane, histogram
                              of unsatisfied time bonds u = (V - Bt)/2 before the
                              exchanges, bin = u*1024/(V+1), V = L*L*L_tau     */

typedef struct {
    uint32_t state; /* 0 never at slot 0, 1 heading up, 2 heading down */
    uint32_t t_last;/* PT time of the last visit to slot 0              */
    uint32_t count; /* completed round trips 0 -> N-1 -> 0               */
    uint32_t pad;
    uint64_t sum;   /* sum of their durations, in PT steps               */
} qsg_roundtrip;

/* Bytes of device workspace needed for these groups (Sec. 2.1: the state of
 * one MCQSG run -- spins of every ladder point, couplings, the precomputed
 * acceptance factors -- here for n_groups groups side by side; App. A: the
 * energy measurement and the PT random walk `history_betas` as per-slot
 * counters, sums, walker labels and a swap log of cfg->swaplog_cap rows).
 * groups: host array of n_groups descriptors; cfg: host run settings; both
 * only read.  Returns 0 on any invalid input, and also for a group of more
 * than 2^29 words per slot (L*L*L_tau > 2^29: the kernels address a slot
 * with 32-bit byte offsets and hold bond sums in 32-bit integers). */
size_t qsg_workspace_bytes(const qsg_group_desc* groups, uint32_t n_groups,
                           const qsg_run_config* cfg);

/* Create a context over `d_workspace` (device pointer, 256-byte aligned,
 * >= qsg_workspace_bytes) on HIP stream `hip_stream` (hipStream_t, may be
 * NULL for the null stream).  Builds the couplings on the device from the
 * lane seeds (App. A: the couplings come from their own seed, separate from
 * the seeds of the initial configuration and of the Monte Carlo numbers;
 * here each lane's J_{i,d} = -1 iff bit 0 of word 0 of Philox4x32-10 with
 * counter (x + L y, d, 3<<24, 0) under key j_seed[lane] is set, Sec. 2.1.1).
 * The ladder is unset until qsg_set_gamma_ladder (or qsg_set_k_ladder for
 * QSG_LADDER_K groups).  groups and cfg are host memory, read only; the
 * workspace stays the caller's and must outlive the context.  *out is set
 * only on success.  QSG_E_INVALID for a malformed descriptor, null or
 * misaligned workspace; QSG_E_UNSUPPORTED for L*L*L_tau > 2^29 or more
 * than 2^31 blocks in one pass; QSG_E_BUFFER if ws_bytes is too small;
 * none of these touches the device. */
qsg_status qsg_create(const qsg_group_desc* groups, uint32_t n_groups,
                      const qsg_run_config* cfg, void* d_workspace,
                      size_t ws_bytes, void* hip_stream, qsg_ctx** out);

/* Set group `group`'s ladder: n_gamma host doubles, > 0, non-decreasing
 * (slot 0 = smallest transverse field; App. A: the number of transverse
 * field values, App. C: the decreasing k list = increasing Gamma).  Builds
 * the precomputed acceptance factors of Sec. 2.1 -- here integer thresholds
 * thr = ceil(2^32 min(1, e^{-dE})) - 1 for the 15 classes (n_s, n_t) of
 * every slot, and exchange thresholds for every possible time-bond change
 * of every adjacent pair -- in binary128 on the host (App. C: the tables
 * are built in 128-bit floating point) and uploads them on the context's
 * stream, synchronising it.  QSG_E_UNSUPPORTED if an exchange table would
 * exceed swap_table_cap; QSG_E_INVALID for a decreasing or non-positive
 * ladder or a group of ladder_kind QSG_LADDER_K (nothing is changed). */
qsg_status qsg_set_gamma_ladder(qsg_ctx* ctx, uint32_t group, const double* gamma);

/* The same for a group of ladder_kind QSG_LADDER_K: n_gamma couplings k_g,
 * > 0, non-increasing (the paper's decreasing k list, App. C; slot 0 has
 * the largest k, i.e. the smallest transverse field).  Metropolis dE =
 * 4 k_g (3 - n_s - n_t); exchange thresholds from e^{-4 m (k_g - k_{g+1})}
 * for B[g+1] - B[g] = -4m with B = Bsp + Bt. */
qsg_status qsg_set_k_ladder(qsg_ctx* ctx, uint32_t group, const double* k);

/* Random initial spins for every group (App. A: the initial configuration
 * has its own seed; here word (site, slot g) = o0 | o1<<32 of Philox4x32-10,
 * Sec. 2.1.1, with counter (site, 0, 2<<24 | g, group_id) under mc_seed).
 * Resets the sweep and PT counters, walkers (walker g at slot g), round
 * trips, sums and histograms.  Enqueued on the context's stream and
 * synchronised; QSG_E_DEVICE if a launch fails (the context is then
 * failed). */
qsg_status qsg_init_spins(qsg_ctx* ctx);

/* n_sweeps sweeps of every group, with the PT steps that fall due (App. A:
 * an elementary step is `ptfr` full-lattice sweeps, each a red then a blue
 * sublattice update, followed by a parallel-tempering update; here ptfr =
 * cfg->pt_every and a PT step follows sweep t when (t+1) % pt_every == 0;
 * Sec. 2.1: checkerboard Metropolis with precomputed acceptance factors and
 * the exchange probability min(1, e^{(c_g - c_{g+1}) D})).  The sweep and PT
 * indices t, p are global per context and persist across calls and
 * checkpoints.  flags: QSG_PLAIN, or QSG_BATCHED optionally with QSG_GRAPH,
 * QSG_FUSED and QSG_NO_PT; every combination gives the same trajectory.
 * Work is enqueued on the context's stream (asynchronous).  QSG_E_INVALID
 * for unknown flags, QSG_E_STATE before a ladder is set for every group or
 * before spins exist.  With a deadline set (qsg_set_deadline; Sec. 3: the
 * MAXTIME alarm that stops a run cleanly), returns QSG_E_INTERRUPTED after
 * the PT chunk during which it passed; the state is then consistent and can
 * be resumed or checkpointed. */
qsg_status qsg_sweep(qsg_ctx* ctx, uint32_t n_sweeps, uint32_t flags);

/* One PT step now (outside the cadence), every group: energies recomputed
 * from the spins, then the exchanges of Sec. 2.1 for pairs g = 0..N-2 in
 * order, each lane independently (lane j's number: word j&3 of Philox with
 * counter (j>>2, p, 1<<24 | g, group_id)), then the accepted lanes'
 * configurations moved between the two slots.  Advances the PT index p
 * only.  Asynchronous on the context's stream; QSG_E_STATE as qsg_sweep. */
qsg_status qsg_pt_swap(qsg_ctx* ctx);

/* Copy a measurement (see QSG_M_*) to host memory (App. A: the online
 * energy measurement and `history_betas`, the state of the PT random walk;
 * App. E, the overlap of two replicas at equal times, tau1 = tau2).  `what`
 * selects one QSG_M_* value; host_out receives the groups' arrays one after
 * another in group order, with the layout given beside each selector.
 * Synchronises the context's stream.  QSG_E_INVALID for an unknown
 * selector or null buffer, QSG_E_BUFFER if `bytes` is too small (nothing is
 * written), QSG_E_STATE for ENERGY/OVERLAP before spins exist. */
qsg_status qsg_measure(qsg_ctx* ctx, uint32_t what, void* host_out, size_t bytes);

/* Spins of one group as host words, n_words = n_gamma * L_tau * L * L, in
 * the layout above ([slot][tau][y][x], bit j = lane j, bit 1 <=> S = -1:
 * App. D's bit convention).  get: synchronises, then copies; QSG_E_BUFFER
 * if n_words is too small.  set: n_words must match exactly (QSG_E_INVALID
 * otherwise); the stored energies and walkers are not recomputed -- the
 * next PT step recomputes the energies from the spins. */
qsg_status qsg_get_spins(qsg_ctx* ctx, uint32_t group, uint64_t* host, size_t n_words);
qsg_status qsg_set_spins(qsg_ctx* ctx, uint32_t group, const uint64_t* host, size_t n_words);

/* Couplings of one group as built on the device (App. A, flagJ = 0: the
 * couplings are generated from their seed): host Jx[L*L], Jy[L*L], index
 * x + L*y, bit j = lane j, bit 1 <=> J = -1.  Synchronises. */
qsg_status qsg_get_couplings(qsg_ctx* ctx, uint32_t group, uint64_t* jx, uint64_t* jy);

/* Full checkpoint (spins, counters, energies, walkers, round trips, sums,
 * logs, and the ladders for a consistency check) to/from a host buffer of
 * qsg_state_bytes(ctx) bytes (App. A: a run is a back-up or a new run).  No
 * random state exists: the generator is counter-based, its counters tied
 * to the lattice update (Sec. 2.1.1), so a resumed run continues the same
 * trajectory.  set: QSG_E_INVALID for a buffer of another context or
 * another ladder (nothing changed).  Both synchronise the stream. */
size_t qsg_state_bytes(const qsg_ctx* ctx);
qsg_status qsg_get_state(qsg_ctx* ctx, void* host, size_t bytes);
qsg_status qsg_set_state(qsg_ctx* ctx, const void* host, size_t bytes);

/* Thresholds of one group as uploaded (Sec. 2.1's precomputed acceptance
 * factors, App. C's 128-bit construction): host arrays thr[N][15] (index
 * n_s*3+n_t), swap_equal[N-1], swap_len[N-1], swap_thr[N-1][swap_table_cap]
 * (entry m-1 of pair g: threshold for a change D = -4m); any pointer may be
 * NULL to skip it.  Synchronises; QSG_E_STATE if the ladder is not set. */
qsg_status qsg_get_tables(qsg_ctx* ctx, uint32_t group, uint32_t* thr,
                          uint8_t* swap_equal, uint32_t* swap_len, uint32_t* swap_thr);

/* Host-only table builder (no device): same arithmetic as
 * qsg_set_gamma_ladder.  swap_thr has room for (n_gamma-1)*cap entries. */
qsg_status qsg_build_tables(double beta, uint32_t L_tau, uint32_t n_gamma,
                            const double* gamma, uint32_t cap, uint32_t* thr,
                            uint8_t* swap_equal, uint32_t* swap_len, uint32_t* swap_thr);

/* Host-only table builder for a coupling ladder: same arithmetic as
 * qsg_set_k_ladder, same output layout as qsg_build_tables. */
qsg_status qsg_build_tables_k(uint32_t n_gamma, const double* k, uint32_t cap, uint32_t* thr,
                              uint8_t* swap_equal, uint32_t* swap_len, uint32_t* swap_thr);

/* Colour-pass schedule of one group (the autotuner's knob; no paper basis:
 * it replaces the paper's threads-per-block argument of Sec. 3): Philox
 * blocks every word goes through before the words still undecided are
 * packed into fewer waves, 1..16 (16 = never).  Results do not depend on
 * it.  Synchronises; QSG_E_INVALID outside 1..16 (nothing changed). */
qsg_status qsg_set_schedule(qsg_ctx* ctx, uint32_t group, uint32_t sweep_split);

/* Both colour-pass knobs of one group: sweep_split as above and tau_tile,
 * the tau planes one thread walks along its column (2..32; the group uses
 * the largest power of two <= tau_tile that divides its L_tau).  The batched
 * launch plan is rebuilt (and a captured graph dropped).  Results do not
 * depend on either knob.  Synchronises; QSG_E_INVALID for values outside
 * their ranges (nothing changed). */
qsg_status qsg_set_colour_schedule(qsg_ctx* ctx, uint32_t group, uint32_t sweep_split,
                                   uint32_t tau_tile);

/* Wall-clock deadline checked between PT chunks of qsg_sweep (Sec. 3: the
 * MAXTIME value that stops a run cleanly before a batch limit): seconds
 * from now; 0: due now, so the next qsg_sweep stops after its first chunk;
 * < 0 clears it.  QSG_E_INVALID for NaN.  Touches no device state. */
qsg_status qsg_set_deadline(qsg_ctx* ctx, double seconds_from_now);

/* Synchronise the context's stream; QSG_E_DEVICE if queued work failed. */
qsg_status qsg_sync(qsg_ctx* ctx);

/* Message of the last failure of this context (or, for NULL, of the last
 * failed creation or context-free call of this thread).  The string is
 * owned by the library and valid until the next call on the context. */
const char* qsg_last_error(const qsg_ctx* ctx);

/* Synchronise, then release the context's host objects and HIP graphs; the
 * caller then frees the workspace.  NULL is ignored. */
void qsg_destroy(qsg_ctx* ctx);

/* Philox4x32-10 on the device, for known-answer checks (Sec. 2.1.1: the
 * paper's generator, Salmon et al.): for i < n, out[4i..] =
 * Philox(ctr = in[6i..6i+3], key = in[6i+4..6i+5]).  Device pointers owned
 * by the caller; asynchronous on hip_stream.  QSG_E_INVALID for null
 * buffers, QSG_E_DEVICE if the launch fails. */
qsg_status qsg_philox(const uint32_t* d_in, uint32_t* d_out, uint32_t n, void* hip_stream);

/* Euclidean-time overlaps of the configurations now in slots first_slot ..
 * first_slot + n_slots - 1 of group `group`, one launch (App. E: the
 * tau-dependent Q2, Q4 and F of `overlap_tau`).  For each slot, with
 * q_x = S(x,tau1) S(x,tau1+tau) (tau1 + tau modulo L_tau), Qt = sum_x q_x,
 * column sums C_x1 = sum over y of q and row sums R_x2 = sum over x of q,
 * adds for every tau = taus[i] (host array, i < n_taus <= 64, tau < L_tau):
 *   q2[a][i] += sum_tau1 Qt^2 and q4[a][i] += sum_tau1 Qt^4 for lane a,
 *   A[i][d] += sum over lanes and tau1 of sum_x1 C_x1 C_{x1+d}, B likewise
 *   with R (d < L, indices modulo L),
 * into d_out (device, caller-owned and caller-zeroed int64, per slot
 * q2 [64][n_taus], q4 [64][n_taus], A [n_taus][L], B [n_taus][L], slots one
 * after the other; out_words >= n_slots * n_taus * (128 + 2L)).  Then
 * Q2(tau) = <q2>/L_tau,
 * Q4(tau) = <q4>/L_tau and F(tau) = sum_d (A+B)(d) cos(2 pi d/L) /
 * (2 * 64 * L_tau) per call.  Integer sums: exact, order-independent.
 * Needs L <= 32 (QSG_E_UNSUPPORTED otherwise).  Enqueued on the context's
 * stream; does not change the chain. */
qsg_status qsg_tau_overlaps(qsg_ctx* ctx, uint32_t group, uint32_t first_slot, uint32_t n_slots,
                            const uint32_t* taus, uint32_t n_taus, int64_t* d_out,
                            size_t out_words);

/* The observables of App. E (`overlap_tau`: Q2, Q4 and F as functions of
 * the Euclidean-time distance) from the integer sums of qsg_tau_overlaps
 * over n_configs configurations of one slot: host arrays q2 [64][n_taus],
 * q4 [64][n_taus], A [n_taus][L], B [n_taus][L] (one slot's block of the
 * overlaps output, summed), averaged over tau1, the configurations and the
 * 64 replicas: Q2[i] = mean_lanes q2 / (L_tau n_configs), likewise Q4, and
 * F[i] = sum_d (A+B)[i][d] cos(2 pi d / L) / (2 * 64 * L_tau * n_configs).
 * Outputs are host arrays of n_taus doubles.  Host only: no device, no
 * context.  QSG_E_INVALID for null pointers, L = 0, L_tau = 0, n_taus = 0
 * or n_configs = 0. */
qsg_status qsg_tau_observables(const int64_t* sums, uint32_t L, uint32_t L_tau, uint32_t n_taus,
                               uint64_t n_configs, double* Q2, double* Q4, double* F);

/* Random-number ceiling of the device (measurement only; the generator of
 * Sec. 2.1.1): thread i < n_threads generates `blocks` Philox4x32-10 blocks
 * with counters (i, 0, b, 0), b < blocks, under key (key lo, key hi) -- the
 * counter shape of the colour pass, one per-thread word -- and writes the xor
 * of all 4*blocks output words to d_out[i] (device, n_threads words, caller
 * owned).  Asynchronous on hip_stream.  Timing it gives Philox blocks per
 * second with nothing else in the way. */
qsg_status qsg_philox_probe(uint32_t n_threads, uint32_t blocks, uint64_t key, uint32_t* d_out,
                            void* hip_stream);

/* ------------------------------------------------------------------------
 * Transfer matrix of one L x L slice in a parity sector (paper: Sec. 2.2,
 * the EDQSG code and its matrix-free product; App. D, the parity-aware
 * basis), float64:
 *   T = W B W,  W = diag exp(k Bsp(n) / 2),
 *   B = prod over the L^2 sites of (jp 1 + jm sigma^X),
 *   jp = e^kp / (e^kp + e^-kp), jm = e^-kp / (e^kp + e^-kp),
 * i.e. the slice transfer matrix of the Trotter-Suzuki form (weight
 * exp(k Bsp + kp Bt) per prism configuration) divided by (2 cosh kp)^(L^2);
 * the paper's equal-coupling form is kp = k.  Sector vectors have
 * qsg_tm_dim(L) = 2^(L^2-1) doubles: entry n is the basis state
 * (|n> + parity |~n>) / sqrt(2), n the spins of sites 0 .. L^2-2 (site
 * j = x1 + L x2, bit j set <=> S_j = -1, the last site +1), ~n the complement
 * of all L^2 bits.  Bsp(n) sums J S S' over the bonds (j, +x) and (j, +y),
 * periodic.  One GPU holds L <= 5 (2^24 doubles per vector); larger L
 * returns QSG_E_UNSUPPORTED.
 * ---------------------------------------------------------------------- */
#define QSG_TM_MAX_L 5

typedef struct {
    uint32_t L;       /* 2 .. QSG_TM_MAX_L */
    int32_t parity;   /* +1 even sector, -1 odd sector */
    double k;         /* space coupling (finite) */
    double k_perp;    /* time coupling (finite) */
    int8_t jx[QSG_TM_MAX_L * QSG_TM_MAX_L];  /* +-1: coupling of bond (j, +x), j < L*L */
    int8_t jy[QSG_TM_MAX_L * QSG_TM_MAX_L];  /* +-1: coupling of bond (j, +y); rest ignored */
} qsg_tm_desc;

/* 2^(L^2-1), or 0 when L is outside 2 .. QSG_TM_MAX_L. */
uint64_t qsg_tm_dim(uint32_t L);

/* d_out = T d_in in the descriptor's sector: qsg_tm_dim(L) doubles each,
 * device memory owned by the caller; d_in == d_out is allowed (other
 * overlaps are not).  Enqueued on hip_stream (one or two kernels);
 * QSG_E_INVALID for a bad descriptor or null pointer, QSG_E_UNSUPPORTED
 * for L > QSG_TM_MAX_L, QSG_E_DEVICE if a launch fails; the message is
 * qsg_last_error(NULL). */
qsg_status qsg_tm_apply(const qsg_tm_desc* d, const double* d_in, double* d_out,
                        void* hip_stream);

/* Device workspace of qsg_tm_lanczos: (max_iter + 2) sector vectors plus
 * small reduction buffers; 0 for an unsupported L or max_iter 0. */
size_t qsg_tm_lanczos_workspace_bytes(uint32_t L, uint32_t max_iter);

/* Largest eigenvalues of the sector's T by the Lanczos method (the paper
 * leaves the iteration to a library; here it runs on the device with full
 * reorthogonalisation, classical Gram-Schmidt applied twice, deterministic
 * reductions).  Start vector: uniform [-1, 1) from splitmix64 of `seed`.
 * Stops after max_iter steps, when the n_eig largest Ritz values all have
 * residual estimates |beta_m y_m| <= tol * |largest|, or when the Krylov
 * space is exhausted (then every Ritz value is exact).  Outputs (host):
 * eigs[n_eig] descending, resid[n_eig] the residual estimates, *iters the
 * steps taken; distinct Ritz values only (a multiple eigenvalue appears
 * once), entries beyond the number found are NaN.  d_vec (device, may be
 * NULL): the unit Ritz vector of eigs[0].  d_ws: qsg_tm_lanczos_workspace_
 * bytes(L, max_iter) bytes, device, caller owned.  Synchronises hip_stream
 * (every step reads two scalars back).  1 <= n_eig <= max_iter <= 4096. */
qsg_status qsg_tm_lanczos(const qsg_tm_desc* d, uint32_t max_iter, uint32_t n_eig, double tol,
                          uint64_t seed, void* d_ws, size_t ws_bytes, double* eigs,
                          double* resid, uint32_t* iters, double* d_vec, void* hip_stream);

/* Ground-state correlation functions (paper: App. E, the consistency checks
 * of EDQSG, L_tau -> infinity): for the sector vector d_vec (qsg_tm_dim(L)
 * doubles, device; normally the leading eigenvector of the even sector,
 * any norm: the weights v_n^2 are normalised), with
 * M_xy = <v| sZ_x sZ_y |v>, R_xyzu = <v| sZ_x sZ_y sZ_z sZ_u |v> and
 * Mt_xy = M_xy [cos(2 pi (x1-y1)/L) + cos(2 pi (x2-y2)/L)] / 2:
 *   out[0] = Q2 = Tr M^2,  out[1] = Q4 = sum_{x,y,z,u} R_xyzu^2,
 *   out[2] = F = Tr M Mt   (host, 3 doubles).
 * Computed from the Walsh-Hadamard transform of v^2 on the device (the
 * product's passes with the factor (a, b) -> (a + b, a - b)) and a
 * fixed-order reduction over the pairs and quadruples of sites.  d_ws:
 * qsg_tm_correlations_workspace_bytes(L) bytes of device memory, caller
 * owned.  Synchronises hip_stream. */
size_t qsg_tm_correlations_workspace_bytes(uint32_t L);
qsg_status qsg_tm_correlations(uint32_t L, const double* d_vec, void* d_ws, size_t ws_bytes,
                               double* out, void* hip_stream);

/* Finite-L_tau estimates of the same correlations (paper: App. E; EDQSG
 * reports them for a list of Euclidean lengths): a slice of the periodic
 * prism of L_tau slices sees the two leading states, the even one d_even
 * with eigenvalue lambda_even and the odd one d_odd with lambda_odd
 * (sector vectors of qsg_tm_dim(L) doubles, device, any norm), mixed with
 * the odd weight w = lambda_odd^L_tau / (lambda_even^L_tau +
 * lambda_odd^L_tau); every correlation of the previous call becomes
 * (1 - w) <e|..|e> + w <o|..|o> before it is squared.  l_taus: n lengths
 * (host), 0 meaning L_tau -> infinity (w = 0, the result of
 * qsg_tm_correlations on d_even).  out: 3n doubles (host), (Q2, Q4, F) per
 * length; 1 <= n <= 4096.  The eigenvalues must be positive and finite
 * (QSG_E_INVALID otherwise).  d_ws: qsg_tm_correlations_lt_workspace_bytes(L, n) bytes of
 * device memory, caller owned.  Synchronises hip_stream. */
size_t qsg_tm_correlations_lt_workspace_bytes(uint32_t L, uint32_t n);
qsg_status qsg_tm_correlations_lt(uint32_t L, const double* d_even, const double* d_odd,
                                  double lambda_even, double lambda_odd, const uint32_t* l_taus,
                                  uint32_t n, void* d_ws, size_t ws_bytes, double* out,
                                  void* hip_stream);

/* ------------------------------------------------------------------------
 * Learned Gamma ladder: a 6 -> 128 -> 128 -> 128 -> 32 MLP (exact-erf GELU on
 * the hidden layers) mapping (L, L_tau, beta, frustrated-plaquette fraction,
 * Gamma_min, Gamma_max) features to 31 increment logits of log Gamma and a
 * log total exchange barrier.  No paper basis: an addition on top of the
 * method that only chooses the ladder the PT step uses (Sec. 2.1).
 * Parameters: qsg_mlp_param_count() FP32 values, flat W1[6][128], b1,
 * W2[128][128], b2, W3[128][128], b3, W4[128][32], b4 (W[k][n] maps input k
 * to output n), plus an optional BF16 copy: when it is given, every GEMM
 * operand is rounded to bfloat16 and products accumulate in FP32.  All
 * pointers are device pointers owned by the caller; work is enqueued on
 * `hip_stream`; results are deterministic.
 * ---------------------------------------------------------------------- */
uint32_t qsg_mlp_param_count(void);

/* Floats of forward workspace for a batch of B (activations kept for the
 * backward pass). */
size_t qsg_mlp_workspace_floats(uint32_t B);

/* out[B][32] = MLP(x[B][6]); ws: qsg_mlp_workspace_floats(B) floats. */
qsg_status qsg_mlp_forward(const float* d_params, const uint16_t* d_params_bf16,
                           const float* d_x, uint32_t B, float* d_out, float* d_ws,
                           void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * forward pass as qsg_mlp_forward, bit for bit, with its workspace in a
 * fixed device array of the library (QSG_MLP_NOALLOC_MAX_BATCH * 800 floats,
 * 3.2 MB, one copy per GPU, held until the process ends) instead of d_ws.
 * The caller passes parameters, inputs and outputs.  No allocation happens
 * in this call.  The array's address is looked up on the first call on each
 * device.  Calls on one GPU share that GPU's array, so calls that overlap
 * on one GPU (other streams, other threads) race; serialise them.
 * QSG_E_INVALID for null pointers, B = 0 or B > QSG_MLP_NOALLOC_MAX_BATCH
 * (nothing is launched); QSG_E_DEVICE if the lookup or a launch fails. */
#define QSG_MLP_NOALLOC_MAX_BATCH 1024
qsg_status qsg_mlp_forward_noalloc(const float* d_params, const uint16_t* d_params_bf16,
                                   const float* d_x, uint32_t B, float* d_out, void* hip_stream);

/* Gradients of a scalar loss w.r.t. the FP32 parameters, given dL/d(out)
 * d_dout[B][32] and the forward workspace of the same batch.
 * d_scratch: 2*B*128 floats.  d_grads: qsg_mlp_param_count() floats. */
qsg_status qsg_mlp_backward(const float* d_params, const uint16_t* d_params_bf16,
                            const float* d_x, const float* d_ws, const float* d_dout,
                            uint32_t B, float* d_grads, float* d_scratch, void* hip_stream);

/* Per sample: KL(t || softmax(z[0..30])) + (z[31] - logL)^2 into d_loss[B],
 * and d_dz[B][32] = gradient of the batch mean. */
qsg_status qsg_mlp_loss(const float* d_z, const float* d_target_inc, const float* d_target_logL,
                        uint32_t B, float* d_dz, float* d_loss, void* hip_stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8; step >= 1) on the FP32
 * parameters; refreshes the BF16 copy when given.  m, v: FP32 moments. */
qsg_status qsg_mlp_adam(float* d_params, uint16_t* d_params_bf16, const float* d_grads,
                        float* d_m, float* d_v, uint32_t step, float lr, void* hip_stream);

/* BF16 copy of the FP32 parameters (nearest even). */
qsg_status qsg_mlp_to_bf16(const float* d_params, uint16_t* d_params_bf16, void* hip_stream);

/* Ladders d_ladder[B][32] (doubles, non-decreasing, ends exactly gmin and
 * gmax) from outputs d_z[B][32]: log G_i = log gmin + (log gmax - log gmin)
 * * sum_{l<i} softmax(z[0..30])_l; d_acc_pred[B] = 1 - exp(z[31])/31 (may be
 * NULL). */
qsg_status qsg_mlp_decode(const float* d_z, const double* d_gmin, const double* d_gmax,
                          uint32_t B, double* d_ladder, float* d_acc_pred, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* QSG_H */
