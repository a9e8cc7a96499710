// C ABI of the MCQSG hot path (declared in include/qsg.h).
//
// The context lives on the host; all device state is carved out of one
// caller-owned workspace.  Plain sweeps launch every kernel once per group
// (one launch per disorder sample, as a per-sample run would); batched
// sweeps launch each pass once over every group, optionally replaying a
// captured HIP graph of one PT chunk (pt_every sweeps, energy pass, PT step,
// exchange pass, counter advance).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/qsg.h"
#include "qsg_internal.h"
#include "qsg_overlaps.h"
#include "qsg_mlp.h"

extern "C" int qsg_tables_build_host(double beta, uint32_t L_tau, uint32_t N, const double* gamma,
                                     uint32_t cap, uint32_t* thr, uint8_t* eq, uint32_t* len,
                                     uint32_t* sw, char* err, size_t errlen);
extern "C" int qsg_tables_build_host_k(uint32_t N, const double* k, uint32_t cap, uint32_t* thr,
                                       uint8_t* eq, uint32_t* len, uint32_t* sw, char* err,
                                       size_t errlen);

static_assert(qsg::kMaxSlots == QSG_MAX_GAMMA, "kernels size per-group arrays by the slot limit");
static_assert(qsg::kMlpNoAllocMaxBatch == QSG_MLP_NOALLOC_MAX_BATCH, "one batch limit for the allocation-free forward");

namespace {

using qsg::GroupDev;
using qsg::RoundTrip;

constexpr size_t kAlign = 256;
constexpr uint32_t kDefaultSwapCap = 4096;
constexpr uint64_t kStateMagic = 0x31544B5043475351ull;  // "QSGCPKT1"

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

thread_local std::string g_create_error;

struct Region {
    size_t off = 0, bytes = 0;
};

// Byte layout of one group inside the workspace.
struct GroupLayout {
    Region spins, Jx, Jy, jseed, thr, sw_thr, sw_len, sw_eq, cnt, meas, E, walker, rt, acc,
        swaplog, sums, lastmask, hist;
};

struct Layout {
    std::vector<GroupLayout> g;
    Region groups_dev, prefix_sweep, prefix_energy, prefix_swap, prefix_slots, counters;
    Region block_map;  // colour-pass block -> (group, block in group), unequal groups only
    size_t total = 0;
};

uint32_t swap_cap_of(const qsg_group_desc& d) {
    return d.swap_table_cap ? d.swap_table_cap : kDefaultSwapCap;
}

// Largest slot, in words: the colour pass addresses a slot as a base pointer
// plus a 32-bit byte offset, and per-lane bond sums and their differences
// are held in 32-bit integers (|Bsp| <= 2V, |Bt| <= V), both exact up to
// V = 2^29 words (4 GiB per slot).
constexpr uint64_t kMaxSlotWords = 1ull << 29;

// QSG_OK, or QSG_E_INVALID for a malformed descriptor, or QSG_E_UNSUPPORTED
// for a well-formed one beyond the slot size the kernels address.
qsg_status check_desc(const qsg_group_desc& d, std::string* why) {
    char buf[256];
    qsg_status code = QSG_E_INVALID;
    if (d.L < 2 || d.L > 256 || (d.L & 1)) {
        std::snprintf(buf, sizeof buf, "L=%u must be even and in [2, 256]", d.L);
    } else if (d.L_tau < 2 || d.L_tau > 65536 || (d.L_tau & 1)) {
        std::snprintf(buf, sizeof buf, "L_tau=%u must be even and in [2, 65536]", d.L_tau);
    } else if (!(d.beta > 0) || d.beta != d.beta || d.beta > 1e300) {
        std::snprintf(buf, sizeof buf, "beta must be finite and > 0");
    } else if (d.n_gamma < 1 || d.n_gamma > QSG_MAX_GAMMA) {
        std::snprintf(buf, sizeof buf, "n_gamma=%u must be in [1, %d]", d.n_gamma, QSG_MAX_GAMMA);
    } else if (d.ladder_kind != QSG_LADDER_GAMMA && d.ladder_kind != QSG_LADDER_K) {
        std::snprintf(buf, sizeof buf, "ladder_kind=%u unknown", d.ladder_kind);
    } else if (d.tau_boundary != QSG_TAU_PERIODIC && d.tau_boundary != QSG_TAU_ANTIPERIODIC) {
        std::snprintf(buf, sizeof buf, "tau_boundary=%u unknown", d.tau_boundary);
    } else if (d.reserved != 0) {
        std::snprintf(buf, sizeof buf, "reserved field must be 0");
    } else if (swap_cap_of(d) > (1u << 24)) {
        std::snprintf(buf, sizeof buf, "swap_table_cap too large");
    } else if ((uint64_t)d.L * d.L * d.L_tau > kMaxSlotWords) {
        std::snprintf(buf, sizeof buf, "L*L*L_tau = %llu words per slot exceeds the limit 2^29",
                      (unsigned long long)d.L * d.L * d.L_tau);
        code = QSG_E_UNSUPPORTED;
    } else {
        return QSG_OK;
    }
    if (why) *why = buf;
    return code;
}

// QSG_OK or the status of the first bad descriptor (with `why` set).
qsg_status make_layout(const qsg_group_desc* d, uint32_t n, const qsg_run_config& cfg,
                       Layout* out, std::string* why) {
    Layout L;
    size_t off = 0;
    auto take = [&off](size_t bytes) {
        Region r;
        r.off = off;
        r.bytes = bytes;
        off = align_up(off + (bytes ? bytes : 1));
        return r;
    };
    L.counters = take(2 * sizeof(uint32_t));
    L.groups_dev = take(sizeof(GroupDev) * n);
    L.prefix_sweep = take(sizeof(uint32_t) * (n + 1));
    L.prefix_energy = take(sizeof(uint32_t) * (n + 1));
    L.prefix_swap = take(sizeof(uint32_t) * (n + 1));
    L.prefix_slots = take(sizeof(uint32_t) * (n + 1));
    for (uint32_t i = 0; i < n; ++i) {
        if (qsg_status st = check_desc(d[i], why)) {
            if (why) *why = "group " + std::to_string(i) + ": " + *why;
            return st;
        }
        const size_t N = d[i].n_gamma, P = (size_t)d[i].L * d[i].L;
        const size_t V = P * d[i].L_tau;
        const size_t pairs = N > 1 ? N - 1 : 1;
        GroupLayout g;
        g.spins = take(N * V * 8);
        g.Jx = take(P * 8);
        g.Jy = take(P * 8);
        g.jseed = take(64 * 8);
        g.thr = take(N * qsg::kThrStride * 4);
        g.sw_thr = take(pairs * swap_cap_of(d[i]) * 4);
        g.sw_len = take(pairs * 4);
        g.sw_eq = take(pairs * 4);
        g.cnt = take(N * qsg::kCntStride * 4);
        g.meas = take(N * qsg::kCntStride * 4);
        g.E = take(N * 64 * 2 * 4);
        g.walker = take(N * 64 * 4);
        g.rt = take(N * 64 * sizeof(RoundTrip));
        g.acc = take(pairs * 8);
        g.swaplog = take((size_t)cfg.swaplog_cap * pairs * 8);
        g.sums = take(N * qsg::kSumStride * 8);
        g.lastmask = take(N * 8);
        g.hist = take(N * qsg::kHistBins * 4);
        L.g.push_back(g);
    }
    // the colour pass's block map, when the groups' block counts differ
    // (sized for the shallowest column walk, which needs the most blocks, so
    // that any schedule set later fits)
    std::vector<uint64_t> blocks(n);
    for (uint32_t i = 0; i < n; ++i)
        blocks[i] = (uint64_t)d[i].n_gamma *
                    qsg::sweep_blocks_per_slot(d[i].L * d[i].L * d[i].L_tau, 2);
    bool equal = true;
    uint64_t total_blocks = 0;
    for (uint32_t i = 0; i < n; ++i) {
        equal = equal && blocks[i] == blocks[0];
        total_blocks += blocks[i];
    }
    // every pass launches one grid over all groups: its block count must be
    // a valid grid size and fit the 32-bit block prefix sums
    uint64_t energy_blocks = 0, swap_blocks = 0;
    for (uint32_t i = 0; i < n; ++i) {
        const uint32_t V = d[i].L * d[i].L * d[i].L_tau;
        energy_blocks += (uint64_t)d[i].n_gamma *
                         qsg::energy_blocks_per_slot(V, qsg::tile_for(d[i].L_tau, qsg::kEnergyWords));
        swap_blocks += qsg::swap_blocks(V);
    }
    if (total_blocks >= (1ull << 31) || energy_blocks >= (1ull << 31) ||
        swap_blocks >= (1ull << 31)) {
        if (why) *why = "the groups together need more than 2^31 blocks in one pass";
        return QSG_E_UNSUPPORTED;
    }
    L.block_map = take(equal ? 0 : total_blocks * sizeof(qsg::BlockEntry));
    L.total = off;
    *out = std::move(L);
    return QSG_OK;
}

// Which specialised class list covers every class of this slot that is not
// accepted outright (threshold below 2^32-1): 0, 1, 2, or 3 for the generic
// fifteen-class update.  The lists match the kernels' Classes<R>.
const int kRegimeLists[3][7][2] = {
    {{0, 0}, {1, 0}, {2, 0}, {3, 0}, {4, 0}, {0, 1}, {1, 1}},
    {{0, 0}, {1, 0}, {2, 0}, {3, 0}, {0, 1}, {1, 1}, {0, 2}},
    {{0, 0}, {1, 0}, {2, 0}, {0, 1}, {1, 1}, {0, 2}, {1, 2}},
};

uint32_t class_regime(const uint32_t* thr15) {
    for (uint32_t r = 0; r < 3; ++r) {
        bool covered = true;
        for (int c = 0; c < 15 && covered; ++c) {
            if (thr15[c] == 0xFFFFFFFFu) continue;
            bool in = false;
            for (int i = 0; i < 7; ++i)
                in |= (kRegimeLists[r][i][0] * 3 + kRegimeLists[r][i][1] == c);
            covered = in;
        }
        if (covered) return r;
    }
    return 3;
}

// Level picks of a slot in regime r < 3: per comparison level (bit 31 - b of
// the thresholds, b = 0..31) the set of the regime's seven classes whose
// threshold bit is 1, or its complement with bit 7 set when that is smaller,
// so the colour pass ORs at most three class masks per level.
void level_picks(const uint32_t* thr15, uint32_t r, uint32_t* out8) {
    for (int w = 0; w < 8; ++w) out8[w] = 0;
    if (r > 2) return;
    for (int b = 0; b < 32; ++b) {
        uint32_t set = 0;
        for (int i = 0; i < 7; ++i) {
            const int c = kRegimeLists[r][i][0] * 3 + kRegimeLists[r][i][1];
            set |= ((thr15[c] >> (31 - b)) & 1u) << i;
        }
        const uint32_t pick = __builtin_popcount(set) > 3 ? ((~set & 0x7Fu) | 0x80u) : set;
        out8[b >> 2] |= pick << (8 * (b & 3));
    }
}

}  // namespace

struct qsg_ctx {
    std::vector<qsg_group_desc> desc;
    qsg_run_config cfg{};
    Layout layout;
    uint8_t* ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr;
    hipStream_t capture_stream = nullptr;
    std::vector<GroupDev> gd;         // host copies of the device group records
    std::vector<std::vector<double>> ladder;
    std::vector<bool> ladder_set;
    uint32_t* d_counters = nullptr;   // device (t, p)
    uint64_t t = 0, p = 0;            // host mirror of the device counters
    qsg::BatchPlan plan_sweep{}, plan_energy{}, plan_swap{};
    GroupDev* d_groups = nullptr;
    qsg::BatchPlan plan_slots{};      // one block per slot (fused sweeps)
    uint32_t fused_lds_words = 0;     // slots at most this big run from LDS
    hipGraphExec_t chunk_exec[2] = {nullptr, nullptr};  // [fused]
    hipGraph_t chunk_graph[2] = {nullptr, nullptr};
    bool failed = false;
    bool spins_ready = false;
    bool has_deadline = false;
    double deadline = 0;  // steady-clock seconds
    std::string err;
};

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

qsg_status fail(qsg_ctx* c, qsg_status code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) {
        c->err = buf;
        if (code == QSG_E_DEVICE) c->failed = true;
    } else {
        g_create_error = buf;
    }
    return code;
}

#define QSG_HIP(c, expr)                                                                   \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail((c), QSG_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

qsg_status check_ctx(qsg_ctx* c) {
    if (!c) return fail(nullptr, QSG_E_INVALID, "null context");
    if (c->failed) return QSG_E_STATE;
    return QSG_OK;
}

template <class T>
T* at(qsg_ctx* c, const Region& r) {
    return reinterpret_cast<T*>(c->ws + r.off);
}

qsg_status check_ready(qsg_ctx* c) {
    for (size_t i = 0; i < c->desc.size(); ++i)
        if (!c->ladder_set[i])
            return fail(c, QSG_E_STATE, "group %zu has no Gamma ladder", i);
    if (!c->spins_ready) return fail(c, QSG_E_STATE, "spins not initialised");
    return QSG_OK;
}

void destroy_graph(qsg_ctx* c) {
    for (int f = 0; f < 2; ++f) {
        if (c->chunk_exec[f]) (void)hipGraphExecDestroy(c->chunk_exec[f]);
        if (c->chunk_graph[f]) (void)hipGraphDestroy(c->chunk_graph[f]);
        c->chunk_exec[f] = nullptr;
        c->chunk_graph[f] = nullptr;
    }
}

// ---------------------------------------------------------------- passes --
qsg_status plain_sweep(qsg_ctx* c, uint32_t t_add) {
    for (const GroupDev& g : c->gd)
        QSG_HIP(c, qsg::launch_half_sweep(g, 0, c->d_counters, t_add, c->stream));
    for (const GroupDev& g : c->gd)
        QSG_HIP(c, qsg::launch_half_sweep(g, 1, c->d_counters, t_add, c->stream));
    return QSG_OK;
}

qsg_status plain_pt(qsg_ctx* c, uint32_t p_add) {
    for (const GroupDev& g : c->gd) {
        QSG_HIP(c, qsg::launch_energy(g, g.cnt, c->stream));
        QSG_HIP(c, qsg::launch_pt(g, c->d_counters, p_add, c->stream));
        QSG_HIP(c, qsg::launch_swap_apply(g, c->stream));
    }
    return QSG_OK;
}

qsg_status batched_sweep(qsg_ctx* c, hipStream_t s, uint32_t t_add) {
    QSG_HIP(c, qsg::launch_half_sweep_batched(c->plan_sweep, 0, c->d_counters, t_add, s));
    QSG_HIP(c, qsg::launch_half_sweep_batched(c->plan_sweep, 1, c->d_counters, t_add, s));
    return QSG_OK;
}

qsg_status batched_pt(qsg_ctx* c, hipStream_t s, uint32_t p_add) {
    QSG_HIP(c, qsg::launch_energy_batched(c->plan_energy, s));
    QSG_HIP(c, qsg::launch_pt_batched(c->d_groups, (uint32_t)c->gd.size(), c->d_counters, p_add, s));
    QSG_HIP(c, qsg::launch_swap_apply_batched(c->plan_swap, s));
    return QSG_OK;
}

// One whole PT chunk on stream s: pt_every sweeps (colour passes over all
// groups, or one fused launch), the energy pass, the PT step, the exchange
// pass and the counter advance.
qsg_status enqueue_chunk(qsg_ctx* c, hipStream_t s, bool fused) {
    const uint32_t pe = c->cfg.pt_every;
    if (fused) {
        QSG_HIP(c, qsg::launch_chunk_fused(c->plan_slots, c->d_counters, pe, c->fused_lds_words, s));
    } else {
        for (uint32_t i = 0; i < pe; ++i)
            if (qsg_status st = batched_sweep(c, s, i)) return st;
    }
    if (qsg_status st = batched_pt(c, s, 0)) return st;
    QSG_HIP(c, qsg::launch_advance(c->d_counters, pe, 1, s));
    return QSG_OK;
}

qsg_status build_chunk_graph(qsg_ctx* c, bool fused) {
    const int f = fused ? 1 : 0;
    if (c->chunk_exec[f]) return QSG_OK;
    hipStream_t s = c->capture_stream;
    QSG_HIP(c, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    qsg_status st = enqueue_chunk(c, s, fused);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(s, &graph);
    if (st != QSG_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return fail(c, QSG_E_DEVICE, "graph capture: %s", hipGetErrorString(e));
    c->chunk_graph[f] = graph;
    QSG_HIP(c, hipGraphInstantiate(&c->chunk_exec[f], graph, nullptr, nullptr, 0));
    return QSG_OK;
}

// The colour pass's batched plan from the groups' current schedules: block
// prefix sums (uploaded), the per-group block count when all groups have
// the same, else the block map (uploaded; its region is sized for the
// schedule that needs the most blocks).  Synchronises the stream.
qsg_status upload_sweep_plan(qsg_ctx* c) {
    const uint32_t n = (uint32_t)c->gd.size();
    std::vector<uint32_t> pre(n + 1, 0);
    for (uint32_t i = 0; i < n; ++i) {
        const GroupDev& g = c->gd[i];
        pre[i + 1] = pre[i] + g.N * qsg::sweep_blocks_per_slot(g.V, g.tile);
    }
    hipStream_t s = c->stream;
    qsg::BatchPlan p = qsg::make_plan(c->d_groups, at<uint32_t>(c, c->layout.prefix_sweep),
                                      pre.data(), n, c->gd.data());
    QSG_HIP(c, hipMemcpyAsync(const_cast<uint32_t*>(p.prefix), pre.data(), 4 * (n + 1),
                              hipMemcpyHostToDevice, s));
    std::vector<qsg::BlockEntry> map;
    if (!p.per_group && c->layout.block_map.bytes) {
        map.reserve(pre[n]);
        for (uint32_t i = 0; i < n; ++i)
            for (uint32_t b = 0; b < pre[i + 1] - pre[i]; ++b) map.push_back({i, b});
        if (map.size() * sizeof(qsg::BlockEntry) > c->layout.block_map.bytes)
            return fail(c, QSG_E_INVALID, "block map of %zu entries exceeds its region", map.size());
        auto* d_map = at<qsg::BlockEntry>(c, c->layout.block_map);
        QSG_HIP(c, hipMemcpyAsync(d_map, map.data(), map.size() * sizeof(qsg::BlockEntry),
                                  hipMemcpyHostToDevice, s));
        p.block_map = d_map;
    }
    QSG_HIP(c, hipStreamSynchronize(s));  // the staging vectors go out of scope
    c->plan_sweep = p;
    return QSG_OK;
}

}  // namespace

// Checkpoint: header, then per group the device regions that carry state.
namespace {
struct CkptHeader {
    uint64_t magic, n_groups, t, p, bytes;
};
template <class F>
void for_state_regions(const qsg_ctx* c, F f) {
    for (size_t i = 0; i < c->gd.size(); ++i) {
        const GroupLayout& gl = c->layout.g[i];
        for (const Region* r : {&gl.spins, &gl.E, &gl.walker, &gl.rt, &gl.acc, &gl.swaplog,
                                &gl.sums, &gl.lastmask, &gl.cnt, &gl.hist})
            f(*r);
    }
}
}  // namespace

namespace {
// Build a group's tables with the host builder of its ladder kind and upload
// them (thresholds, regime, level picks, exchange tables).
qsg_status set_ladder(qsg_ctx* c, uint32_t group, const double* values, uint32_t kind) {
    if (qsg_status st = check_ctx(c)) return st;
    if (group >= c->desc.size()) return fail(c, QSG_E_INVALID, "group %u out of range", group);
    if (!values) return fail(c, QSG_E_INVALID, "ladder is null");
    const qsg_group_desc& d = c->desc[group];
    if (d.ladder_kind != kind)
        return fail(c, QSG_E_INVALID, "group %u has ladder kind %u", group, d.ladder_kind);
    const GroupDev& g = c->gd[group];
    const uint32_t N = d.n_gamma, pairs = N > 1 ? N - 1 : 1;
    std::vector<uint32_t> thr15(N * 15), thr(N * qsg::kThrStride, 0), len(pairs, 0),
        sw((size_t)pairs * g.sw_cap, 0), eq32(pairs, 0);
    std::vector<uint8_t> eq(pairs, 0);
    char err[256] = {0};
    int rc = kind == QSG_LADDER_K
                 ? qsg_tables_build_host_k(N, values, g.sw_cap, thr15.data(), eq.data(), len.data(),
                                           sw.data(), err, sizeof err)
                 : qsg_tables_build_host(d.beta, d.L_tau, N, values, g.sw_cap, thr15.data(),
                                         eq.data(), len.data(), sw.data(), err, sizeof err);
    if (rc == -1) return fail(c, QSG_E_INVALID, "%s", err);
    if (rc != 0) return fail(c, QSG_E_UNSUPPORTED, "%s", err);
    for (uint32_t i = 0; i < N; ++i) {
        for (int k = 0; k < 15; ++k) thr[i * qsg::kThrStride + k] = thr15[i * 15 + k];
        const uint32_t r = class_regime(&thr15[i * 15]);
        thr[i * qsg::kThrStride + 15] = r;
        level_picks(&thr15[i * 15], r, &thr[i * qsg::kThrStride + qsg::kLevelPicks]);
    }
    for (uint32_t i = 0; i < pairs; ++i) eq32[i] = eq[i];
    hipStream_t s = c->stream;
    QSG_HIP(c, hipMemcpyAsync(g.thr, thr.data(), thr.size() * 4, hipMemcpyHostToDevice, s));
    QSG_HIP(c, hipMemcpyAsync(g.sw_thr, sw.data(), sw.size() * 4, hipMemcpyHostToDevice, s));
    QSG_HIP(c, hipMemcpyAsync(g.sw_len, len.data(), len.size() * 4, hipMemcpyHostToDevice, s));
    QSG_HIP(c, hipMemcpyAsync(g.sw_eq, eq32.data(), eq32.size() * 4, hipMemcpyHostToDevice, s));
    QSG_HIP(c, hipStreamSynchronize(s));
    c->ladder[group].assign(values, values + N);
    c->ladder_set[group] = true;
    return QSG_OK;
}

}  // namespace

// ====================================================================== ABI
extern "C" {

size_t qsg_workspace_bytes(const qsg_group_desc* groups, uint32_t n_groups,
                           const qsg_run_config* cfg) {
    if (!groups || n_groups == 0 || !cfg || cfg->swaplog_cap == 0 ||
        cfg->tau_tile > qsg::kMaxTile || cfg->tau_tile == 1)
        return 0;
    Layout L;
    std::string why;
    if (make_layout(groups, n_groups, *cfg, &L, &why) != QSG_OK) return 0;
    return L.total;
}

qsg_status qsg_create(const qsg_group_desc* groups, uint32_t n_groups, const qsg_run_config* cfg,
                      void* d_workspace, size_t ws_bytes, void* hip_stream, qsg_ctx** out) {
    if (!out) return fail(nullptr, QSG_E_INVALID, "out is null");
    *out = nullptr;
    if (!groups || n_groups == 0 || !cfg)
        return fail(nullptr, QSG_E_INVALID, "groups/cfg null or n_groups == 0");
    if (cfg->swaplog_cap == 0) return fail(nullptr, QSG_E_INVALID, "swaplog_cap must be >= 1");
    if (cfg->tau_tile > qsg::kMaxTile || cfg->tau_tile == 1)
        return fail(nullptr, QSG_E_INVALID, "tau_tile %u outside 2..%u (0: default)", cfg->tau_tile,
                    qsg::kMaxTile);
    if (!d_workspace || ((uintptr_t)d_workspace % kAlign) != 0)
        return fail(nullptr, QSG_E_INVALID, "workspace must be non-null and 256-byte aligned");
    Layout L;
    std::string why;
    if (qsg_status st = make_layout(groups, n_groups, *cfg, &L, &why))
        return fail(nullptr, st, "%s", why.c_str());
    if (ws_bytes < L.total)
        return fail(nullptr, QSG_E_BUFFER, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);

    qsg_ctx* c = new qsg_ctx();
    c->desc.assign(groups, groups + n_groups);
    c->cfg = *cfg;
    c->layout = L;
    c->ws = static_cast<uint8_t*>(d_workspace);
    c->ws_bytes = ws_bytes;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->ladder.resize(n_groups);
    c->ladder_set.assign(n_groups, false);
    c->d_counters = at<uint32_t>(c, L.counters);
    c->d_groups = at<GroupDev>(c, L.groups_dev);

    std::vector<uint32_t> pre_energy(n_groups + 1, 0),
        pre_swap(n_groups + 1, 0), pre_slots(n_groups + 1, 0);
    uint32_t max_v = 0;
    for (uint32_t i = 0; i < n_groups; ++i) {
        const qsg_group_desc& d = groups[i];
        const GroupLayout& gl = L.g[i];
        GroupDev g{};
        g.L = d.L;
        g.Ltau = d.L_tau;
        g.N = d.n_gamma;
        g.gid = d.group_id;
        g.key0 = (uint32_t)(d.mc_seed & 0xFFFFFFFFu);
        g.key1 = (uint32_t)(d.mc_seed >> 32);
        g.V = d.L * d.L * d.L_tau;
        g.div_half_plane = qsg::make_divisor(d.L * d.L / 2);
        g.div_half_row = qsg::make_divisor(d.L / 2);
        g.div_plane = qsg::make_divisor(d.L * d.L);
        g.div_row = qsg::make_divisor(d.L);
        g.tile = qsg::tile_for(d.L_tau, cfg->tau_tile ? cfg->tau_tile : qsg::kDefaultTile);
        g.etile = qsg::tile_for(d.L_tau, qsg::kEnergyWords);
        g.div_blocks = qsg::make_divisor(qsg::sweep_blocks_per_slot(g.V, g.tile));
        g.sw_cap = swap_cap_of(d);
        g.log_cap = cfg->swaplog_cap;
        g.q_split = cfg->sweep_split ? (cfg->sweep_split > 16 ? 16 : cfg->sweep_split) : 4;
        g.exch_all = d.ladder_kind == QSG_LADDER_K ? 1u : 0u;
        g.anti = d.tau_boundary == QSG_TAU_ANTIPERIODIC ? 1u : 0u;
        g.spins = at<uint64_t>(c, gl.spins);
        g.Jx = at<uint64_t>(c, gl.Jx);
        g.Jy = at<uint64_t>(c, gl.Jy);
        g.jseed = at<uint64_t>(c, gl.jseed);
        g.thr = at<uint32_t>(c, gl.thr);
        g.sw_thr = at<uint32_t>(c, gl.sw_thr);
        g.sw_len = at<uint32_t>(c, gl.sw_len);
        g.sw_eq = at<uint32_t>(c, gl.sw_eq);
        g.cnt = at<int32_t>(c, gl.cnt);
        g.meas = at<int32_t>(c, gl.meas);
        g.E = at<int32_t>(c, gl.E);
        g.walker = at<uint32_t>(c, gl.walker);
        g.rt = at<RoundTrip>(c, gl.rt);
        g.acc = at<uint64_t>(c, gl.acc);
        g.swaplog = at<uint64_t>(c, gl.swaplog);
        g.sums = at<int64_t>(c, gl.sums);
        g.lastmask = at<uint64_t>(c, gl.lastmask);
        g.hist = at<uint32_t>(c, gl.hist);
        c->gd.push_back(g);
        pre_energy[i + 1] = pre_energy[i] + g.N * qsg::energy_blocks_per_slot(g.V, g.etile);
        pre_swap[i + 1] = pre_swap[i] + (g.N >= 2 ? qsg::swap_blocks(g.V) : 0);
        pre_slots[i + 1] = pre_slots[i] + g.N;
        if (g.V > max_v) max_v = g.V;
    }
    c->plan_energy = qsg::make_plan(c->d_groups, at<uint32_t>(c, L.prefix_energy),
                                    pre_energy.data(), n_groups, c->gd.data());
    c->plan_swap = qsg::make_plan(c->d_groups, at<uint32_t>(c, L.prefix_swap), pre_swap.data(),
                                  n_groups, c->gd.data());
    c->plan_slots = qsg::make_plan(c->d_groups, at<uint32_t>(c, L.prefix_slots), pre_slots.data(),
                                   n_groups, c->gd.data());
    c->fused_lds_words = max_v <= qsg::kFusedLdsMaxWords ? max_v : 0;

    auto bail = [&](qsg_status st) {
        g_create_error = c->err;
        delete c;
        return st;
    };
    hipStream_t s = c->stream;
#define CREATE_HIP(expr)                                                                 \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess) {                                                          \
            fail(c, QSG_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));        \
            return bail(QSG_E_DEVICE);                                                   \
        }                                                                                \
    } while (0)
    CREATE_HIP(hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
    CREATE_HIP(hipMemcpyAsync(c->d_groups, c->gd.data(), sizeof(GroupDev) * n_groups,
                              hipMemcpyHostToDevice, s));
    CREATE_HIP(hipMemcpyAsync(const_cast<uint32_t*>(c->plan_energy.prefix), pre_energy.data(), 4 * (n_groups + 1),
                              hipMemcpyHostToDevice, s));
    CREATE_HIP(hipMemcpyAsync(const_cast<uint32_t*>(c->plan_swap.prefix), pre_swap.data(), 4 * (n_groups + 1),
                              hipMemcpyHostToDevice, s));
    CREATE_HIP(hipMemcpyAsync(const_cast<uint32_t*>(c->plan_slots.prefix), pre_slots.data(),
                              4 * (n_groups + 1), hipMemcpyHostToDevice, s));
    if (qsg_status st = upload_sweep_plan(c)) return bail(st);
    const uint32_t zero2[2] = {0, 0};
    CREATE_HIP(hipMemcpyAsync(c->d_counters, zero2, sizeof zero2, hipMemcpyHostToDevice, s));
    for (uint32_t i = 0; i < n_groups; ++i) {
        CREATE_HIP(hipMemcpyAsync(const_cast<uint64_t*>(c->gd[i].jseed), groups[i].j_seed,
                                  64 * 8, hipMemcpyHostToDevice, s));
        CREATE_HIP(qsg::launch_init_couplings(c->gd[i], s));
        CREATE_HIP(qsg::launch_init_state(c->gd[i], s));
    }
    CREATE_HIP(hipStreamSynchronize(s));  // host staging buffers go out of scope
#undef CREATE_HIP
    *out = c;
    return QSG_OK;
}

qsg_status qsg_set_gamma_ladder(qsg_ctx* c, uint32_t group, const double* gamma) {
    return set_ladder(c, group, gamma, QSG_LADDER_GAMMA);
}

qsg_status qsg_set_k_ladder(qsg_ctx* c, uint32_t group, const double* k) {
    return set_ladder(c, group, k, QSG_LADDER_K);
}

qsg_status qsg_init_spins(qsg_ctx* c) {
    if (qsg_status st = check_ctx(c)) return st;
    hipStream_t s = c->stream;
    for (const GroupDev& g : c->gd) {
        QSG_HIP(c, qsg::launch_init_spins(g, s));
        QSG_HIP(c, qsg::launch_init_state(g, s));
    }
    const uint32_t zero2[2] = {0, 0};
    QSG_HIP(c, hipMemcpyAsync(c->d_counters, zero2, sizeof zero2, hipMemcpyHostToDevice, s));
    QSG_HIP(c, hipStreamSynchronize(s));
    c->t = c->p = 0;
    c->spins_ready = true;
    return QSG_OK;
}

qsg_status qsg_sweep(qsg_ctx* c, uint32_t n_sweeps, uint32_t flags) {
    if (qsg_status st = check_ctx(c)) return st;
    if (flags & ~(QSG_BATCHED | QSG_GRAPH | QSG_NO_PT | QSG_FUSED))
        return fail(c, QSG_E_INVALID, "unknown flags 0x%x", flags);
    if ((flags & (QSG_GRAPH | QSG_FUSED)) && !(flags & QSG_BATCHED))
        return fail(c, QSG_E_INVALID, "QSG_GRAPH and QSG_FUSED need QSG_BATCHED");
    if (qsg_status st = check_ready(c)) return st;
    const bool batched = flags & QSG_BATCHED;
    const bool do_pt = !(flags & QSG_NO_PT) && c->cfg.pt_every > 0;
    const uint32_t pe = c->cfg.pt_every;
    uint32_t done = 0;
    while (done < n_sweeps) {
        // whole PT chunks aligned to the cadence: one fused launch for the
        // sweeps and/or a replay of the captured chunk graph
        const bool fused = flags & QSG_FUSED;
        if (batched && (flags & (QSG_GRAPH | QSG_FUSED)) && do_pt && pe > 0 && c->t % pe == 0 &&
            n_sweeps - done >= pe) {
            if (flags & QSG_GRAPH) {
                if (qsg_status st = build_chunk_graph(c, fused)) return st;
                QSG_HIP(c, hipGraphLaunch(c->chunk_exec[fused ? 1 : 0], c->stream));
            } else if (qsg_status st = enqueue_chunk(c, c->stream, fused)) {
                return st;
            }
            done += pe;
            c->t += pe;
            c->p += 1;
        } else {
            // sweeps up to the next PT step (or the end of the request)
            uint32_t n = n_sweeps - done;
            if (do_pt && pe > 0) {
                const uint32_t to_pt = pe - (uint32_t)(c->t % pe);
                if (to_pt < n) n = to_pt;
            }
            for (uint32_t i = 0; i < n; ++i) {
                qsg_status st = batched ? batched_sweep(c, c->stream, i) : plain_sweep(c, i);
                if (st) return st;
            }
            const bool pt_now = do_pt && pe > 0 && (c->t + n) % pe == 0;
            if (pt_now) {
                QSG_HIP(c, qsg::launch_advance(c->d_counters, n, 0, c->stream));
                qsg_status st = batched ? batched_pt(c, c->stream, 0) : plain_pt(c, 0);
                if (st) return st;
                QSG_HIP(c, qsg::launch_advance(c->d_counters, 0, 1, c->stream));
                c->p += 1;
            } else {
                QSG_HIP(c, qsg::launch_advance(c->d_counters, n, 0, c->stream));
            }
            done += n;
            c->t += n;
        }
        if (c->has_deadline && done < n_sweeps) {
            if (now_s() >= c->deadline) {
                QSG_HIP(c, hipStreamSynchronize(c->stream));
                return fail(c, QSG_E_INTERRUPTED, "deadline reached after %u sweeps", done);
            }
        }
    }
    return QSG_OK;
}

qsg_status qsg_pt_swap(qsg_ctx* c) {
    if (qsg_status st = check_ctx(c)) return st;
    if (qsg_status st = check_ready(c)) return st;
    if (qsg_status st = batched_pt(c, c->stream, 0)) return st;
    QSG_HIP(c, qsg::launch_advance(c->d_counters, 0, 1, c->stream));
    c->p += 1;
    return QSG_OK;
}

qsg_status qsg_measure(qsg_ctx* c, uint32_t what, void* host_out, size_t bytes) {
    if (qsg_status st = check_ctx(c)) return st;
    if (!host_out) return fail(c, QSG_E_INVALID, "host_out is null");
    size_t need = 0;
    for (const auto& d : c->desc) {
        const size_t N = d.n_gamma, pairs = N > 1 ? N - 1 : 1;
        switch (what) {
            case QSG_M_ENERGY: need += N * 64 * 2 * 4; break;
            case QSG_M_OVERLAP: need += N * 32 * 8; break;
            case QSG_M_ACCEPT: need += pairs * 8; break;
            case QSG_M_WALKERS: need += N * 64; break;
            case QSG_M_SWAPLOG: need += (size_t)c->cfg.swaplog_cap * pairs * 8; break;
            case QSG_M_ROUNDTRIP: need += N * 64 * sizeof(qsg_roundtrip); break;
            case QSG_M_SUMS: need += N * qsg::kSumStride * 8; break;
            case QSG_M_HIST: need += N * qsg::kHistBins * 4; break;
            case QSG_M_COUNTERS: need = 16; break;
            default: return fail(c, QSG_E_INVALID, "unknown measurement %u", what);
        }
    }
    if (bytes < need) return fail(c, QSG_E_BUFFER, "measure needs %zu bytes, got %zu", need, bytes);
    hipStream_t s = c->stream;
    if (what == QSG_M_COUNTERS) {
        uint64_t v[2] = {c->t, c->p};
        std::memcpy(host_out, v, sizeof v);
        return QSG_OK;
    }
    if (what == QSG_M_ENERGY || what == QSG_M_OVERLAP) {
        if (!c->spins_ready) return fail(c, QSG_E_STATE, "spins not initialised");
        for (const GroupDev& g : c->gd) {
            QSG_HIP(c, qsg::launch_zero32(g.meas, (size_t)g.N * qsg::kCntStride, s));
            QSG_HIP(c, qsg::launch_energy(g, g.meas, s));
        }
        uint8_t* o = static_cast<uint8_t*>(host_out);
        std::vector<int32_t> cnt;
        QSG_HIP(c, hipStreamSynchronize(s));
        for (const GroupDev& g : c->gd) {
            cnt.resize((size_t)g.N * qsg::kCntStride);
            QSG_HIP(c, hipMemcpy(cnt.data(), g.meas, cnt.size() * 4, hipMemcpyDeviceToHost));
            const int64_t V = g.V;
            if (what == QSG_M_ENERGY) {
                int32_t* e = reinterpret_cast<int32_t*>(o);
                for (uint32_t k = 0; k < g.N; ++k)
                    for (int j = 0; j < 64; ++j) {
                        e[(k * 64 + j) * 2 + 0] = (int32_t)(2 * V - 2 * cnt[k * qsg::kCntStride + j]);
                        e[(k * 64 + j) * 2 + 1] = (int32_t)(V - 2 * cnt[k * qsg::kCntStride + 64 + j]);
                    }
                o += (size_t)g.N * 64 * 2 * 4;
            } else {
                int64_t* q = reinterpret_cast<int64_t*>(o);
                for (uint32_t k = 0; k < g.N; ++k)
                    for (int p = 0; p < 32; ++p)
                        q[k * 32 + p] = V - 2 * (int64_t)cnt[k * qsg::kCntStride + 128 + p];
                o += (size_t)g.N * 32 * 8;
            }
        }
        return QSG_OK;
    }
    QSG_HIP(c, hipStreamSynchronize(s));
    uint8_t* o = static_cast<uint8_t*>(host_out);
    for (const GroupDev& g : c->gd) {
        const size_t N = g.N, pairs = N > 1 ? N - 1 : 1;
        switch (what) {
            case QSG_M_ACCEPT:
                QSG_HIP(c, hipMemcpy(o, g.acc, pairs * 8, hipMemcpyDeviceToHost));
                o += pairs * 8;
                break;
            case QSG_M_WALKERS: {
                std::vector<uint32_t> w(N * 64);
                QSG_HIP(c, hipMemcpy(w.data(), g.walker, w.size() * 4, hipMemcpyDeviceToHost));
                for (size_t i = 0; i < w.size(); ++i) o[i] = (uint8_t)w[i];
                o += N * 64;
                break;
            }
            case QSG_M_SWAPLOG:
                QSG_HIP(c, hipMemcpy(o, g.swaplog, (size_t)g.log_cap * pairs * 8,
                                     hipMemcpyDeviceToHost));
                o += (size_t)g.log_cap * pairs * 8;
                break;
            case QSG_M_ROUNDTRIP:
                QSG_HIP(c, hipMemcpy(o, g.rt, N * 64 * sizeof(RoundTrip), hipMemcpyDeviceToHost));
                o += N * 64 * sizeof(RoundTrip);
                break;
            case QSG_M_SUMS:
                QSG_HIP(c, hipMemcpy(o, g.sums, N * qsg::kSumStride * 8, hipMemcpyDeviceToHost));
                o += N * qsg::kSumStride * 8;
                break;
            case QSG_M_HIST:
                QSG_HIP(c, hipMemcpy(o, g.hist, N * qsg::kHistBins * 4, hipMemcpyDeviceToHost));
                o += N * qsg::kHistBins * 4;
                break;
        }
    }
    return QSG_OK;
}

qsg_status qsg_get_spins(qsg_ctx* c, uint32_t group, uint64_t* host, size_t n_words) {
    if (qsg_status st = check_ctx(c)) return st;
    if (group >= c->gd.size() || !host) return fail(c, QSG_E_INVALID, "bad group or buffer");
    const GroupDev& g = c->gd[group];
    const size_t need = (size_t)g.N * g.V;
    if (n_words < need) return fail(c, QSG_E_BUFFER, "need %zu words", need);
    QSG_HIP(c, hipStreamSynchronize(c->stream));
    QSG_HIP(c, hipMemcpy(host, g.spins, need * 8, hipMemcpyDeviceToHost));
    return QSG_OK;
}

qsg_status qsg_set_spins(qsg_ctx* c, uint32_t group, const uint64_t* host, size_t n_words) {
    if (qsg_status st = check_ctx(c)) return st;
    if (group >= c->gd.size() || !host) return fail(c, QSG_E_INVALID, "bad group or buffer");
    const GroupDev& g = c->gd[group];
    const size_t need = (size_t)g.N * g.V;
    if (n_words != need) return fail(c, QSG_E_INVALID, "need exactly %zu words", need);
    QSG_HIP(c, hipStreamSynchronize(c->stream));
    QSG_HIP(c, hipMemcpy(g.spins, host, need * 8, hipMemcpyHostToDevice));
    c->spins_ready = true;
    return QSG_OK;
}

qsg_status qsg_get_couplings(qsg_ctx* c, uint32_t group, uint64_t* jx, uint64_t* jy) {
    if (qsg_status st = check_ctx(c)) return st;
    if (group >= c->gd.size() || !jx || !jy) return fail(c, QSG_E_INVALID, "bad group or buffer");
    const GroupDev& g = c->gd[group];
    QSG_HIP(c, hipStreamSynchronize(c->stream));
    QSG_HIP(c, hipMemcpy(jx, g.Jx, (size_t)g.L * g.L * 8, hipMemcpyDeviceToHost));
    QSG_HIP(c, hipMemcpy(jy, g.Jy, (size_t)g.L * g.L * 8, hipMemcpyDeviceToHost));
    return QSG_OK;
}


size_t qsg_state_bytes(const qsg_ctx* c) {
    if (!c) return 0;
    size_t n = sizeof(CkptHeader);
    for (size_t i = 0; i < c->desc.size(); ++i) n += c->desc[i].n_gamma * sizeof(double);
    for_state_regions(c, [&n](const Region& r) { n += r.bytes; });
    return n;
}

qsg_status qsg_get_state(qsg_ctx* c, void* host, size_t bytes) {
    if (qsg_status st = check_ctx(c)) return st;
    const size_t need = qsg_state_bytes(c);
    if (!host) return fail(c, QSG_E_INVALID, "host is null");
    if (bytes < need) return fail(c, QSG_E_BUFFER, "state needs %zu bytes", need);
    QSG_HIP(c, hipStreamSynchronize(c->stream));
    uint8_t* o = static_cast<uint8_t*>(host);
    CkptHeader h{kStateMagic, c->gd.size(), c->t, c->p, need};
    std::memcpy(o, &h, sizeof h);
    o += sizeof h;
    for (size_t i = 0; i < c->desc.size(); ++i) {
        const size_t n = c->desc[i].n_gamma * sizeof(double);
        if (c->ladder_set[i]) std::memcpy(o, c->ladder[i].data(), n);
        else std::memset(o, 0, n);
        o += n;
    }
    hipError_t err = hipSuccess;
    for_state_regions(c, [&](const Region& r) {
        if (err == hipSuccess) err = hipMemcpy(o, c->ws + r.off, r.bytes, hipMemcpyDeviceToHost);
        o += r.bytes;
    });
    if (err != hipSuccess) return fail(c, QSG_E_DEVICE, "state copy: %s", hipGetErrorString(err));
    return QSG_OK;
}

qsg_status qsg_set_state(qsg_ctx* c, const void* host, size_t bytes) {
    if (qsg_status st = check_ctx(c)) return st;
    const size_t need = qsg_state_bytes(c);
    if (!host || bytes < need) return fail(c, QSG_E_INVALID, "state buffer too small or null");
    const uint8_t* in = static_cast<const uint8_t*>(host);
    CkptHeader h;
    std::memcpy(&h, in, sizeof h);
    if (h.magic != kStateMagic || h.n_groups != c->gd.size() || h.bytes != need)
        return fail(c, QSG_E_INVALID, "checkpoint does not match this context");
    const uint8_t* q = in + sizeof h;
    for (size_t i = 0; i < c->desc.size(); ++i) {
        const size_t n = c->desc[i].n_gamma * sizeof(double);
        if (!c->ladder_set[i] || std::memcmp(q, c->ladder[i].data(), n) != 0)
            return fail(c, QSG_E_INVALID, "group %zu: ladder differs from the checkpoint's", i);
        q += n;
    }
    QSG_HIP(c, hipStreamSynchronize(c->stream));
    hipError_t err = hipSuccess;
    for_state_regions(c, [&](const Region& r) {
        if (err == hipSuccess) err = hipMemcpy(c->ws + r.off, q, r.bytes, hipMemcpyHostToDevice);
        q += r.bytes;
    });
    if (err != hipSuccess) return fail(c, QSG_E_DEVICE, "state copy: %s", hipGetErrorString(err));
    const uint32_t ctr[2] = {(uint32_t)h.t, (uint32_t)h.p};
    QSG_HIP(c, hipMemcpy(c->d_counters, ctr, sizeof ctr, hipMemcpyHostToDevice));
    c->t = h.t;
    c->p = h.p;
    c->spins_ready = true;
    return QSG_OK;
}

qsg_status qsg_get_tables(qsg_ctx* c, uint32_t group, uint32_t* thr, uint8_t* swap_equal,
                          uint32_t* swap_len, uint32_t* swap_thr) {
    if (qsg_status st = check_ctx(c)) return st;
    if (group >= c->gd.size()) return fail(c, QSG_E_INVALID, "group out of range");
    if (!c->ladder_set[group]) return fail(c, QSG_E_STATE, "ladder not set");
    const GroupDev& g = c->gd[group];
    const uint32_t N = g.N, pairs = N > 1 ? N - 1 : 1;
    QSG_HIP(c, hipStreamSynchronize(c->stream));
    if (thr) {
        std::vector<uint32_t> t16((size_t)N * qsg::kThrStride);
        QSG_HIP(c, hipMemcpy(t16.data(), g.thr, t16.size() * 4, hipMemcpyDeviceToHost));
        for (uint32_t i = 0; i < N; ++i)
            for (int k = 0; k < 15; ++k) thr[i * 15 + k] = t16[i * qsg::kThrStride + k];
    }
    if (swap_equal && N > 1) {
        std::vector<uint32_t> e(pairs);
        QSG_HIP(c, hipMemcpy(e.data(), g.sw_eq, pairs * 4, hipMemcpyDeviceToHost));
        for (uint32_t i = 0; i < N - 1; ++i) swap_equal[i] = (uint8_t)e[i];
    }
    if (swap_len && N > 1)
        QSG_HIP(c, hipMemcpy(swap_len, g.sw_len, (N - 1) * 4, hipMemcpyDeviceToHost));
    if (swap_thr && N > 1)
        QSG_HIP(c, hipMemcpy(swap_thr, g.sw_thr, (size_t)(N - 1) * g.sw_cap * 4,
                             hipMemcpyDeviceToHost));
    return QSG_OK;
}

qsg_status qsg_build_tables(double beta, uint32_t L_tau, uint32_t n_gamma, const double* gamma,
                            uint32_t cap, uint32_t* thr, uint8_t* swap_equal, uint32_t* swap_len,
                            uint32_t* swap_thr) {
    if (n_gamma == 0 || n_gamma > QSG_MAX_GAMMA || !gamma || cap == 0)
        return fail(nullptr, QSG_E_INVALID, "bad n_gamma, gamma or cap");
    char err[256] = {0};
    int rc = qsg_tables_build_host(beta, L_tau, n_gamma, gamma, cap, thr, swap_equal, swap_len,
                                   swap_thr, err, sizeof err);
    if (rc == -1) return fail(nullptr, QSG_E_INVALID, "%s", err);
    if (rc != 0) return fail(nullptr, QSG_E_UNSUPPORTED, "%s", err);
    return QSG_OK;
}

qsg_status qsg_build_tables_k(uint32_t n_gamma, const double* k, uint32_t cap, uint32_t* thr,
                              uint8_t* swap_equal, uint32_t* swap_len, uint32_t* swap_thr) {
    if (n_gamma == 0 || n_gamma > QSG_MAX_GAMMA || !k || cap == 0)
        return fail(nullptr, QSG_E_INVALID, "bad n_gamma, k or cap");
    char err[256] = {0};
    int rc = qsg_tables_build_host_k(n_gamma, k, cap, thr, swap_equal, swap_len, swap_thr, err,
                                     sizeof err);
    if (rc == -1) return fail(nullptr, QSG_E_INVALID, "%s", err);
    if (rc != 0) return fail(nullptr, QSG_E_UNSUPPORTED, "%s", err);
    return QSG_OK;
}

// qsg::same_but_identity lists every field of the group record and the
// kernels' group_record moves every pointer: a new field must be added to
// both.
static_assert(sizeof(GroupDev) == 14 * 4 + 5 * sizeof(qsg::Divisor) + 18 * sizeof(void*),
              "GroupDev changed: update same_but_identity and group_record");

qsg_status qsg_set_colour_schedule(qsg_ctx* c, uint32_t group, uint32_t sweep_split,
                                   uint32_t tau_tile) {
    if (qsg_status st = check_ctx(c)) return st;
    if (group >= c->gd.size()) return fail(c, QSG_E_INVALID, "group %u out of range", group);
    if (sweep_split < 1 || sweep_split > 16)
        return fail(c, QSG_E_INVALID, "sweep_split %u outside 1..16", sweep_split);
    if (tau_tile < 2 || tau_tile > qsg::kMaxTile)
        return fail(c, QSG_E_INVALID, "tau_tile %u outside 2..%u", tau_tile, qsg::kMaxTile);
    GroupDev& g = c->gd[group];
    const GroupDev before = g;
    g.q_split = sweep_split;
    g.tile = qsg::tile_for(g.Ltau, tau_tile);
    g.div_blocks = qsg::make_divisor(qsg::sweep_blocks_per_slot(g.V, g.tile));
    // later launches (and the next graph capture) see the new record, in
    // device memory and in the plans' copies
    hipError_t e = hipMemcpyAsync(c->d_groups + group, &g, sizeof(GroupDev),
                                  hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        g = before;
        return fail(c, QSG_E_DEVICE, "schedule upload: %s", hipGetErrorString(e));
    }
    const uint32_t n = (uint32_t)c->gd.size();
    if (qsg_status st = upload_sweep_plan(c)) return st;
    for (qsg::BatchPlan* p : {&c->plan_energy, &c->plan_swap, &c->plan_slots})
        qsg::set_plan_shape(*p, c->gd.data(), n);
    destroy_graph(c);
    return QSG_OK;
}

qsg_status qsg_set_schedule(qsg_ctx* c, uint32_t group, uint32_t sweep_split) {
    if (qsg_status st = check_ctx(c)) return st;
    if (group >= c->gd.size()) return fail(c, QSG_E_INVALID, "group %u out of range", group);
    return qsg_set_colour_schedule(c, group, sweep_split, c->gd[group].tile);
}

qsg_status qsg_set_deadline(qsg_ctx* c, double seconds_from_now) {
    if (!c) return fail(nullptr, QSG_E_INVALID, "null context");
    if (seconds_from_now != seconds_from_now) return fail(c, QSG_E_INVALID, "deadline is NaN");
    c->has_deadline = seconds_from_now >= 0;
    c->deadline = c->has_deadline ? now_s() + seconds_from_now : 0;
    return QSG_OK;
}

qsg_status qsg_sync(qsg_ctx* c) {
    if (qsg_status st = check_ctx(c)) return st;
    QSG_HIP(c, hipStreamSynchronize(c->stream));
    return QSG_OK;
}

const char* qsg_last_error(const qsg_ctx* c) {
    return c ? c->err.c_str() : g_create_error.c_str();
}

void qsg_destroy(qsg_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    destroy_graph(c);
    if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    delete c;
}

qsg_status qsg_philox(const uint32_t* d_in, uint32_t* d_out, uint32_t n, void* hip_stream) {
    if (!d_in || !d_out) return fail(nullptr, QSG_E_INVALID, "null buffer");
    hipError_t e = qsg::launch_philox(d_in, d_out, n, static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return fail(nullptr, QSG_E_DEVICE, "philox launch: %s", hipGetErrorString(e));
    return QSG_OK;
}

qsg_status qsg_tau_overlaps(qsg_ctx* c, uint32_t group, uint32_t first_slot, uint32_t n_slots,
                            const uint32_t* taus, uint32_t n_taus, int64_t* d_out,
                            size_t out_words) {
    if (qsg_status st = check_ctx(c)) return st;
    if (group >= c->gd.size()) return fail(c, QSG_E_INVALID, "group %u out of range", group);
    const GroupDev& g = c->gd[group];
    if (n_slots == 0 || first_slot >= g.N || n_slots > g.N - first_slot)
        return fail(c, QSG_E_INVALID, "slots %u..%u out of range", first_slot,
                    first_slot + n_slots);
    if (g.L > qsg::kOvMaxL)
        return fail(c, QSG_E_UNSUPPORTED, "tau overlaps need L <= %u", qsg::kOvMaxL);
    if (!taus || n_taus == 0 || n_taus > qsg::kOvMaxTaus)
        return fail(c, QSG_E_INVALID, "need 1..%u tau values", qsg::kOvMaxTaus);
    qsg::TauList tl{};
    tl.n = n_taus;
    for (uint32_t i = 0; i < n_taus; ++i) {
        if (taus[i] >= g.Ltau) return fail(c, QSG_E_INVALID, "tau %u >= L_tau", taus[i]);
        tl.t[i] = taus[i];
    }
    const size_t need = (size_t)n_slots * n_taus * (2 * 64 + 2 * g.L);
    if (!d_out) return fail(c, QSG_E_INVALID, "output is null");
    if (out_words < need) return fail(c, QSG_E_BUFFER, "output needs %zu int64", need);
    QSG_HIP(c, qsg::launch_tau_overlaps(g.spins + (size_t)first_slot * g.V, n_slots, g.L, g.Ltau,
                                        tl, d_out, c->stream));
    return QSG_OK;
}

qsg_status qsg_tau_observables(const int64_t* sums, uint32_t L, uint32_t L_tau, uint32_t n_taus,
                               uint64_t n_configs, double* Q2, double* Q4, double* F) {
    if (!sums || !Q2 || !Q4 || !F) return fail(nullptr, QSG_E_INVALID, "null buffer");
    if (L == 0 || L_tau == 0 || n_taus == 0 || n_configs == 0)
        return fail(nullptr, QSG_E_INVALID, "L, L_tau, n_taus and n_configs must be > 0");
    const int64_t* q2 = sums;
    const int64_t* q4 = q2 + (size_t)64 * n_taus;
    const int64_t* A = q4 + (size_t)64 * n_taus;
    const int64_t* B = A + (size_t)n_taus * L;
    const double norm = (double)L_tau * (double)n_configs;
    const double pi = 3.14159265358979323846;
    for (uint32_t i = 0; i < n_taus; ++i) {
        double s2 = 0.0, s4 = 0.0, f = 0.0;
        for (uint32_t a = 0; a < 64; ++a) {  // lane order, as the average is defined
            s2 += (double)q2[(size_t)a * n_taus + i];
            s4 += (double)q4[(size_t)a * n_taus + i];
        }
        for (uint32_t d = 0; d < L; ++d)
            f += (double)(A[(size_t)i * L + d] + B[(size_t)i * L + d]) * std::cos(2.0 * pi * d / L);
        Q2[i] = s2 / 64.0 / norm;
        Q4[i] = s4 / 64.0 / norm;
        F[i] = f / (2.0 * norm * 64.0);
    }
    return QSG_OK;
}

qsg_status qsg_philox_probe(uint32_t n_threads, uint32_t blocks, uint64_t key, uint32_t* d_out,
                            void* hip_stream) {
    if (!d_out && n_threads) return fail(nullptr, QSG_E_INVALID, "null buffer");
    hipError_t e = qsg::launch_philox_probe(d_out, n_threads, blocks, key,
                                            static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return fail(nullptr, QSG_E_DEVICE, "philox probe launch: %s", hipGetErrorString(e));
    return QSG_OK;
}

uint32_t qsg_mlp_param_count(void) { return (uint32_t)qsg::kMlpParams; }

size_t qsg_mlp_workspace_floats(uint32_t B) { return qsg::mlp_ws_floats((int)B); }

static qsg_status mlp_status(hipError_t e, const char* what) {
    if (e != hipSuccess) return fail(nullptr, QSG_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
    return QSG_OK;
}

static bool mlp_batch_ok(uint32_t B) { return B >= 1 && B <= (1u << 20); }

qsg_status qsg_mlp_forward(const float* d_params, const uint16_t* d_params_bf16, const float* d_x,
                           uint32_t B, float* d_out, float* d_ws, void* hip_stream) {
    if (!d_params || !d_x || !d_out || !d_ws || !mlp_batch_ok(B))
        return fail(nullptr, QSG_E_INVALID, "mlp_forward: null buffer or bad batch");
    return mlp_status(qsg::mlp_forward(d_params, d_params_bf16, d_x, (int)B, d_out, d_ws,
                                       static_cast<hipStream_t>(hip_stream)),
                      "mlp_forward");
}

qsg_status qsg_mlp_forward_noalloc(const float* d_params, const uint16_t* d_params_bf16,
                                   const float* d_x, uint32_t B, float* d_out, void* hip_stream) {
    if (!d_params || !d_x || !d_out || B < 1)
        return fail(nullptr, QSG_E_INVALID, "mlp_forward_noalloc: null buffer or empty batch");
    if (B > (uint32_t)qsg::kMlpNoAllocMaxBatch)
        return fail(nullptr, QSG_E_INVALID, "mlp_forward_noalloc: batch %u exceeds the limit %d",
                    B, qsg::kMlpNoAllocMaxBatch);
    return mlp_status(qsg::mlp_forward_noalloc(d_params, d_params_bf16, d_x, (int)B, d_out,
                                               static_cast<hipStream_t>(hip_stream)),
                      "mlp_forward_noalloc");
}

qsg_status qsg_mlp_backward(const float* d_params, const uint16_t* d_params_bf16, const float* d_x,
                            const float* d_ws, const float* d_dout, uint32_t B, float* d_grads,
                            float* d_scratch, void* hip_stream) {
    if (!d_params || !d_x || !d_ws || !d_dout || !d_grads || !d_scratch || !mlp_batch_ok(B))
        return fail(nullptr, QSG_E_INVALID, "mlp_backward: null buffer or bad batch");
    return mlp_status(qsg::mlp_backward(d_params, d_params_bf16, d_x, d_ws, d_dout, (int)B, d_grads,
                                        d_scratch, static_cast<hipStream_t>(hip_stream)),
                      "mlp_backward");
}

qsg_status qsg_mlp_loss(const float* d_z, const float* d_target_inc, const float* d_target_logL,
                        uint32_t B, float* d_dz, float* d_loss, void* hip_stream) {
    if (!d_z || !d_target_inc || !d_target_logL || !d_dz || !d_loss || !mlp_batch_ok(B))
        return fail(nullptr, QSG_E_INVALID, "mlp_loss: null buffer or bad batch");
    return mlp_status(qsg::mlp_loss(d_z, d_target_inc, d_target_logL, (int)B, d_dz, d_loss,
                                    static_cast<hipStream_t>(hip_stream)),
                      "mlp_loss");
}

qsg_status qsg_mlp_adam(float* d_params, uint16_t* d_params_bf16, const float* d_grads, float* d_m,
                        float* d_v, uint32_t step, float lr, void* hip_stream) {
    if (!d_params || !d_grads || !d_m || !d_v || step == 0 || !(lr >= 0))
        return fail(nullptr, QSG_E_INVALID, "mlp_adam: null buffer, step 0 or bad lr");
    return mlp_status(qsg::mlp_adam(d_params, d_params_bf16, d_grads, d_m, d_v, step, lr,
                                    static_cast<hipStream_t>(hip_stream)),
                      "mlp_adam");
}

qsg_status qsg_mlp_to_bf16(const float* d_params, uint16_t* d_params_bf16, void* hip_stream) {
    if (!d_params || !d_params_bf16) return fail(nullptr, QSG_E_INVALID, "mlp_to_bf16: null buffer");
    return mlp_status(qsg::mlp_to_bf16(d_params, d_params_bf16, static_cast<hipStream_t>(hip_stream)),
                      "mlp_to_bf16");
}

qsg_status qsg_mlp_decode(const float* d_z, const double* d_gmin, const double* d_gmax, uint32_t B,
                          double* d_ladder, float* d_acc_pred, void* hip_stream) {
    if (!d_z || !d_gmin || !d_gmax || !d_ladder || !mlp_batch_ok(B))
        return fail(nullptr, QSG_E_INVALID, "mlp_decode: null buffer or bad batch");
    return mlp_status(qsg::mlp_decode(d_z, d_gmin, d_gmax, (int)B, d_ladder, d_acc_pred,
                                      static_cast<hipStream_t>(hip_stream)),
                      "mlp_decode");
}

}  // extern "C"

namespace qsg {
// Failure of a context-free entry point: recorded for qsg_last_error(NULL).
qsg_status report_error(qsg_status code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_create_error = buf;
    return code;
}
}  // namespace qsg
