"""Benchmark of the MCQSG Metropolis + parallel-tempering hot path on one GPU.

Default workload: the batched uneven ensemble, 256 disorder samples (one
group of 64 replicas each) with L in {8,12,16,20,24}, L_tau in
{64,128,256}, beta = L_tau/16 and 24-48 Gammas geometric in [2, 4], PT
every 10 sweeps; seeded synthetic couplings and spins.  A step is one PT
chunk over every sample: 10 sweeps (red + blue pass each), the
energy/overlap pass, the PT step and the exchange pass.

Prints one JSON line.  value = picoseconds per spin-update of the batched
path (one launch per pass over all samples, replayed as a HIP graph, the
faster of the per-pass and fused forms; colour-pass schedules tuned first:
one walk depth for the ensemble, a split per shape class);
plain_ps_per_spin_update is the same work launched per sample, at the walk
depth best for per-sample launches.  The other
half of the metric, PT round trips per hour with the learned against the
geometric ladder, is measured by `python -m paper_2402_03920_amd.learn_ladder`
(profiles/ladder_eval_results.txt); the line quotes that record.
Other modes print their own line: --overlaps (Euclidean-time overlaps),
--transfer (transfer-matrix product and Lanczos), --mlp (ladder network
kernels), --copy-calibration (a plain copy for scaling HBM counters).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# VALU issue peak in lane-instructions per second: 256 CUs x 4 SIMDs x 16
# lanes x 2.4 GHz (a wave64 instruction occupies a SIMD for four cycles; the
# 32-bit integer instructions used here, v_mad_u64_u32 included, all issue at
# that rate)
PEAK_VALU_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# HBM bytes a colour pass must move per updated word: every word of the slot
# is read once (the updated colour and its neighbours, 2 x 8 B per updated
# word) and the updated word is written (8 B)
BYTES_PER_UPDATED_WORD = 24
# fewest gfx950 VALU instructions for one Philox4x32-10 block per lane:
# 10 rounds x (2 v_mad_u64_u32 + 2 three-input xors)
INSTR_PER_PHILOX_BLOCK = 40


def required_blocks_per_word(lanes: int = 64) -> float:
    """Expected Philox blocks the bit-sliced MSB-first comparison needs for a
    word whose `lanes` lanes are all undecided: a lane is decided at each
    level with probability 1/2 and a block carries two levels, so the count
    is E[ceil(M/2)] with M the largest of `lanes` geometric(1/2) levels."""
    return sum(1.0 - (1.0 - 4.0 ** (-(k - 1))) ** lanes for k in range(1, 17))


KERNEL_SOURCES = ("paper_2402_03920_amd/csrc/qsg_kernels.hip",
                  "paper_2402_03920_amd/csrc/qsg_internal.h")
# committed rocprofv3 FETCH_SIZE / WRITE_SIZE summaries of the colour pass,
# per workload
TRAFFIC_FILES = {w: os.path.join(ROOT, "profiles", f"sweep_{w.replace('-', '_')}_traffic.txt")
                 for w in ("uneven", "plain-large", "production")}
TM_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "transfer_l5_traffic.txt")
TM_SOURCES = ("paper_2402_03920_amd/csrc/qsg_transfer.hip",
              "paper_2402_03920_amd/csrc/qsg_transfer.h")
TRAFFIC_RECORDS = [(f, KERNEL_SOURCES) for f in TRAFFIC_FILES.values()] + \
    [(TM_TRAFFIC_FILE, TM_SOURCES)]
LADDER_RECORD = os.path.join(ROOT, "profiles", "ladder_eval_results.txt")


def kernel_source_hash(sources=KERNEL_SOURCES) -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in sources:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic_record(path: str, sources):
    """Fields of a committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary
    (bytes scaled by a plain copy's counters), or None when it is missing or
    was taken on other kernel sources."""
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != kernel_source_hash(sources):
        return None
    return vals


def workload_traffic_record(workload: str):
    """The colour pass's committed traffic and counter summary for this
    workload, or None (none committed, or taken on other kernel sources)."""
    path = TRAFFIC_FILES.get(workload)
    return traffic_record(path, KERNEL_SOURCES) if path else None


def measured_traffic(workload: str):
    """HBM bytes per launch of the colour pass on the bench workload, or
    None (no current summary for this workload)."""
    vals = workload_traffic_record(workload)
    try:
        return int(vals["fetch_bytes_per_launch"]) + int(vals["write_bytes_per_launch"])
    except (TypeError, KeyError, ValueError):
        return None


def ladder_record():
    """Round trips per hour, learned against geometric ladder, from the
    committed evaluation record (not measured by this run)."""
    if not os.path.exists(LADDER_RECORD):
        return None
    out = {"source": os.path.relpath(LADDER_RECORD, ROOT),
           "command": "python -m paper_2402_03920_amd.learn_ladder"}
    section = None
    with open(LADDER_RECORD) as f:
        for line in f:
            if line.startswith("# full evaluation"):
                section = "full"
            elif line.startswith("# focused"):
                section = "focused"
            elif section and line.startswith("round trips per hour"):
                v = line.split(")")[-1].split()
                out[section] = {"geometric": float(v[0]), "learned": float(v[1])}
            elif section and line.startswith("paired round-trip gain"):
                out[section]["paired_gain_per_sample"] = line.split(":", 1)[1].strip()
    return out


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--plain-steps", type=int, default=5)
    ap.add_argument("--samples", type=int, default=64)
    ap.add_argument("--workload", default="uneven",
                    choices=["plain-small", "plain-large", "uneven", "production", "k-ladder"],
                    help="uneven (default): 256 samples of mixed shapes, batched against "
                         "per-sample launches; plain-large: 64 samples, L=16, L_tau=128, "
                         "32 Gammas; plain-small: one sample, L=8, L_tau=32; production: L=24, "
                         "L_tau=2048, 128 samples; k-ladder: the plain-large shape with the "
                         "paper's coupling ladder (PT over k)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default colour-pass schedule instead of tuning it per shape")
    ap.add_argument("--schedules", metavar="JSON",
                    help="take the colour-pass schedules from this file (written by "
                         "--save-schedules) instead of tuning them")
    ap.add_argument("--save-schedules", metavar="JSON",
                    help="write the schedules used to this file (for profiling runs)")
    ap.add_argument("--cpu-sweeps", type=int, default=0,
                    help="oracle sweeps for the CPU baseline (0: about 15 s of work)")
    ap.add_argument("--overlaps", action="store_true",
                    help="time the Euclidean-time overlap measurement instead (one JSON line)")
    ap.add_argument("--transfer", action="store_true",
                    help="time the transfer-matrix product (L = 5 sector) and a Lanczos solve "
                         "instead (one JSON line)")
    ap.add_argument("--mlp", action="store_true",
                    help="time the ladder network's kernels (forward, training step) instead "
                         "(one JSON line)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (to scale HBM counters)")
    return ap.parse_args()


def copy_calibration(mib: int) -> None:
    """A plain device-to-device copy of known size: under rocprofv3 its
    FETCH_SIZE / WRITE_SIZE give the factor that turns the counters of the
    sweep kernels into bytes."""
    import torch
    n = mib << 20
    src = torch.ones(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_launch": n, "launches": 3}), flush=True)


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(groups are independent; sharding them needs no communication)",
              file=sys.stderr)
        sys.exit(2)
    if args.overlaps:
        overlap_bench(args)
        return
    if args.transfer:
        transfer_bench(args)
        return
    if args.mlp:
        mlp_bench(args)
        return
    import numpy as np
    import torch

    import qsg_workloads as W
    from paper_2402_03920_amd import autotune, qsg

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    wl = W.plain_large(n_samples=args.samples) if args.workload == "plain-large" else \
        W.ALL[args.workload]()
    pe = wl.pt_every
    upd_per_sweep = wl.spin_updates_per_sweep()
    words_per_sweep = sum(g.words for g in wl.groups)

    schedules = {}
    if args.schedules:
        schedules = autotune.load_cache(args.schedules)
    elif not args.no_autotune:
        print("[bench] tuning the colour-pass schedule per shape", file=sys.stderr, flush=True)
        schedules = autotune.tune(wl.groups, log=lambda m: print(m, file=sys.stderr, flush=True))
    if args.save_schedules:
        autotune.save_cache(schedules, args.save_schedules)
    ens = qsg.Ensemble(wl.groups, pt_every=pe, swaplog_cap=64)
    if schedules:
        autotune.apply(ens, schedules)
    ens.init_spins()
    stream = ens.stream

    def timed(fn):
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / 1e3

    # the two batched forms of a PT chunk, both replayed as a HIP graph: one
    # launch per colour pass over every group, or one fused launch for all the
    # sweeps of the chunk (a block per slot); the faster one is the value
    form, flags, probe = autotune.pick_form(ens)
    forms = autotune.FORMS
    print(f"[bench] warmup {args.warmup} steps", file=sys.stderr, flush=True)
    ens.sweep(pe * args.warmup, flags)
    torch.cuda.synchronize()
    print(f"[bench] timing {args.steps} batched steps ({form})", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    sec = timed(lambda: ens.sweep(pe * args.steps, flags))
    wall = time.perf_counter() - t0
    ps_batched = sec / (pe * args.steps * upd_per_sweep) * 1e12
    other = [n for n in forms if n != form][0]
    sec_other = timed(lambda: ens.sweep(pe * args.plain_steps, forms[other]))
    ps_other = sec_other / (pe * args.plain_steps * upd_per_sweep) * 1e12

    # per-sample launches: their own walk depth (they fill the chip one group
    # at a time), then back to the batched schedules
    plain_tile, _ = autotune.pick_plain_tile(ens, schedules)
    print(f"[bench] timing {args.plain_steps} plain steps (walk depth {plain_tile})",
          file=sys.stderr, flush=True)
    sec_plain = timed(lambda: ens.sweep(pe * args.plain_steps, qsg.QSG_PLAIN))
    ps_plain = sec_plain / (pe * args.plain_steps * upd_per_sweep) * 1e12
    for i, g in enumerate(ens.groups):
        ens.set_schedule(i, *schedules.get(autotune.shape_key(g), autotune.DEFAULT))

    # dominant kernel: the batched colour pass; average launch duration from
    # events around sweeps without PT (two pass launches + one tiny counter
    # update per sweep), on the stream the kernels run on
    n_k = 2 * pe
    sec_k = timed(lambda: ens.sweep(n_k, qsg.QSG_BATCHED | qsg.QSG_NO_PT))
    pass_s = sec_k / (2 * n_k)
    words_per_pass = words_per_sweep / 2
    blocks = required_blocks_per_word()
    ops_per_pass = words_per_pass * blocks * INSTR_PER_PHILOX_BLOCK
    achieved = ops_per_pass / pass_s / 1e12
    t, p = ens.counters()
    physics = summarize(wl, ens)
    ens.close()
    ceiling = philox_ceiling()
    traffic = measured_traffic(args.workload)

    result = {
        "metric": "ps/spin-update (1 GPU) batched vs plain",
        "value": round(ps_batched, 5),
        "unit": "ps/spin-update",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sec / args.steps * 1e3, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {
            "workload": describe(wl, args.workload),
            "step": f"{pe} sweeps + energy pass + PT step + exchange pass, all samples",
            "spin_updates_per_step": upd_per_sweep * pe,
            "batched_form": form,
            "form_ms_per_chunk": {k: round(v * 1e3, 4) for k, v in probe.items()},
            "schedules": schedules,
        },
        f"{other}_ps_per_spin_update": round(ps_other, 5),
        "plain_ps_per_spin_update": round(ps_plain, 5),
        "plain_tau_tile": plain_tile,
        "batched_speedup_vs_plain": round(ps_plain / ps_batched, 4),
        "spin_updates_per_s": upd_per_sweep * pe * args.steps / sec,
        "wall_s_timed_region": round(wall, 4),
        "roofline": {
            "bound": "alu",
            "kernel": "k_half_sweep_batched",
            "achieved": round(achieved, 4),
            "peak": round(PEAK_VALU_TOPS, 4),
            "unit": "T VALU lane-instructions/s",
            "frac": round(achieved / PEAK_VALU_TOPS, 4),
            "traffic": traffic,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "algorithmic_bytes_per_launch": int(words_per_pass * BYTES_PER_UPDATED_WORD),
            "avg_launch_us": round(pass_s * 1e6, 3),
            "algorithmic_ops_per_launch": ops_per_pass,
            "model": f"required Philox work only: {blocks:.4f} blocks/word x "
                     f"{INSTR_PER_PHILOX_BLOCK} instr x {int(words_per_pass)} words/launch",
            "hbm_GBps_algorithmic": round(words_per_pass * BYTES_PER_UPDATED_WORD / pass_s / 1e9, 2),
        },
    }
    required_rate = words_per_pass * blocks / pass_s
    if traffic is not None:
        result["roofline"]["hbm_GBps_measured"] = round(traffic / pass_s / 1e9, 2)
        result["roofline"]["hbm_frac_measured"] = round(traffic / pass_s / 8e12, 4)
        rec = workload_traffic_record(args.workload)
        try:  # every VALU instruction the kernel issues (counters), not only the required ones
            executed = float(rec["valu_instr_per_wave"]) * float(rec["waves_per_launch"]) * 64
            result["roofline"]["executed_valu_frac"] = round(executed / pass_s / 1e12 / PEAK_VALU_TOPS, 4)
        except (TypeError, KeyError, ValueError):
            pass
    result["philox_ceiling"] = dict(ceiling, sweep_required_blocks_per_s=required_rate,
                                    sweep_frac_of_ceiling=round(required_rate / ceiling["blocks_per_s"], 4))
    result["physics"] = physics
    result["pt_roundtrips_per_hour"] = ladder_record()
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(wl, args.cpu_sweeps)
    print(json.dumps(result), flush=True)


def overlap_bench(args):
    """Time qsg_tau_overlaps on the bench workload's first sample: every slot,
    14 tau values, after a few sweeps; the kernel is VALU-bound, about
    5 L^2 instructions per (tau1, tau) pair and wave (64 replicas)."""
    import numpy as np
    import torch
    import qsg_workloads as W
    from paper_2402_03920_amd import qsg
    torch.cuda.set_device(0)
    g = W.plain_large(n_samples=1).groups[0]
    taus = sorted(set(int(x) for x in np.unique(np.geomspace(1, g.L_tau - 1, 15).astype(int))) | {0})
    import ctypes as C
    t = np.ascontiguousarray(np.asarray(taus, dtype=np.uint32))
    words = len(g.gammas) * len(taus) * (128 + 2 * g.L)
    with qsg.Ensemble([g], pt_every=10, swaplog_cap=8) as ens:
        ens.init_spins()
        ens.sweep(20, qsg.QSG_BATCHED)
        out = torch.zeros(words, dtype=torch.int64, device="cuda")
        ptr = C.c_void_p(out.data_ptr())

        def launch_all():  # every slot of the sample in one launch
            rc = qsg.lib().qsg_tau_overlaps(ens.ctx, 0, 0, len(g.gammas), t.ctypes.data,
                                            len(taus), ptr, words)
            if rc != qsg.QSG_OK:
                raise qsg.QSGError(rc, "tau overlaps")

        launch_all()  # warm-up
        ens.sync()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(ens.stream)
        launch_all()
        b.record(ens.stream)
        torch.cuda.synchronize()
        sec = a.elapsed_time(b) / 1e3
    pairs = len(g.gammas) * len(taus) * g.L_tau
    model = (5.0 * g.L * g.L + 2.0 * g.L) * 64 * pairs  # lane-instructions
    print(json.dumps({"metric": "tau-overlap measurement time", "value": round(sec * 1e3, 4),
                      "unit": "ms per sample (all slots)", "higher_is_better": False,
                      "config": {"workload": f"1 sample, L={g.L}, L_tau={g.L_tau}, "
                                             f"{len(g.gammas)} slots, {len(taus)} tau values"},
                      "us_per_slot_and_tau": round(sec * 1e6 / (len(g.gammas) * len(taus)), 3),
                      "roofline": {"bound": "alu", "model": "5 L^2 + 2 L VALU per (tau1, tau) "
                                   "pair and wave of 64 replicas: per site a bit extraction (2) "
                                   "and two counts, per lag two multiply-adds over half the lags",
                                   "achieved": round(model / sec / 1e12, 4),
                                   "peak": round(PEAK_VALU_TOPS, 4),
                                   "unit": "T VALU lane-instructions/s",
                                   "frac": round(model / sec / 1e12 / PEAK_VALU_TOPS, 4)},
                      "note": "HIP events around one launch over all slots on the library's stream"}),
          flush=True)


def mlp_bench(args):
    """Time the ladder network's kernels (6 -> 128 -> 128 -> 128 -> 32, one
    thread per output, FP32 accumulation) at batch sizes from one sample to
    the allocation-free limit: the forward pass with FP32 and with BF16
    operands, and one training step (forward, loss, backward, Adam), with
    HIP events around back-to-back calls on one stream.  Work per sample:
    2 x (6*128 + 2*128*128 + 128*32) = 75 264 flops forward."""
    import numpy as np
    import torch
    from paper_2402_03920_amd import ladder, qsg
    torch.cuda.set_device(0)
    flops_fwd = 2 * (6 * 128 + 2 * 128 * 128 + 128 * 32)
    reps = max(args.steps, 20)
    s = torch.cuda.current_stream()

    def timed(fn):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(s)
        for _ in range(reps):
            fn()
        b.record(s)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / 1e3 / reps

    rows = []
    rng = np.random.default_rng(11)
    for B in (1, 32, 128, 1024):
        x = torch.tensor(rng.normal(size=(B, 6)).astype(np.float32), device="cuda")
        t_inc = torch.full((B, 31), 1.0 / 31, dtype=torch.float32, device="cuda")
        t_log = torch.zeros(B, dtype=torch.float32, device="cuda")
        row = {"batch": B}
        for name, bf16 in (("fp32", False), ("bf16", True)):
            net = ladder.LadderMLP(seed=3, bf16=bf16)
            ws = torch.empty(int(qsg.lib().qsg_mlp_workspace_floats(B)), dtype=torch.float32,
                             device="cuda")
            out = torch.empty((B, 32), dtype=torch.float32, device="cuda")
            sec = timed(lambda: qsg.qsg_mlp_forward(net.params, net.bf16, x, out, ws))
            row[f"forward_{name}_us"] = round(sec * 1e6, 2)
            row[f"forward_{name}_gflops"] = round(flops_fwd * B / sec / 1e9, 2)
        net = ladder.LadderMLP(seed=3, bf16=True)
        sec = timed(lambda: net.train_step(x, t_inc, t_log, 1e-4))
        row["train_step_us"] = round(sec * 1e6, 2)
        rows.append(row)
    print(json.dumps({"metric": "ladder network kernels", "unit": "us per call",
                      "higher_is_better": False, "reps": reps, "rows": rows,
                      "note": "one thread per output, FP32 accumulation; latency-bound at "
                              "these sizes (a training step is a handful of launches)"}),
          flush=True)


def transfer_bench(args):
    """Time the transfer-matrix product of one L = 5 slice in the even sector
    (2^24 doubles; two passes, each reading and writing the vector once)
    with HIP events around `steps` back-to-back products on one stream, and
    one Lanczos solve for the two largest even eigenvalues.  Algorithmic HBM
    traffic of a product: the input read once and the output written once,
    16 B per sector state."""
    import numpy as np
    import torch
    import qsg_workloads as W
    from paper_2402_03920_amd import qsg
    torch.cuda.set_device(0)
    case = W.transfer_case()
    N = qsg.tm_dim(case.L)
    d = qsg.tm_desc(case.L, case.k, case.k_perp, case.jx, case.jy, 1)
    x = torch.from_numpy(case.vector(0)).cuda()
    y = torch.empty_like(x)
    s = torch.cuda.Stream()
    reps = max(args.steps, 10)
    for _ in range(max(args.warmup, 1)):
        qsg.tm_apply(d, x, y, s)
    s.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(s)
    for _ in range(reps):
        qsg.tm_apply(d, x, y, s)
    b.record(s)
    torch.cuda.synchronize()
    sec = a.elapsed_time(b) / 1e3 / reps
    alg = 16.0 * N
    rec = traffic_record(TM_TRAFFIC_FILE, TM_SOURCES)
    try:
        tm_traffic = int(rec["fetch_bytes_per_product"]) + int(rec["write_bytes_per_product"])
    except (TypeError, KeyError, ValueError):
        tm_traffic = None
    t0 = time.perf_counter()
    lz = qsg.tm_lanczos(d, 300, 2, 1e-9, seed=5, want_vector=True, stream=s)
    lanczos_s = time.perf_counter() - t0
    qsg.tm_correlations(case.L, lz["vector"], stream=s)  # warm-up
    t0 = time.perf_counter()
    corr = qsg.tm_correlations(case.L, lz["vector"], stream=s)
    corr_s = time.perf_counter() - t0
    result = {"metric": "transfer-matrix product time", "value": round(sec * 1e6, 3),
              "unit": "us per product", "higher_is_better": False, "steps": reps,
              "dtype": "f64", "data": "synthetic",
              "config": {"workload": f"transfer-l5: L={case.L} slice, even sector of 2^24 states, "
                                     f"k = k_perp = {case.k}, J = +-1 seed {case.seed}"},
              "roofline": {"bound": "hbm", "kernel": "k_tm_first<true> + k_tm_hi12 (one product)",
                           "achieved": round(alg / sec / 1e9, 2), "peak": 8000.0,
                           "unit": "GB/s", "frac": round(alg / sec / 8e12, 4),
                           "traffic": tm_traffic,
                           "traffic_unit": "HBM bytes per product (rocprofv3 FETCH_SIZE + "
                                           "WRITE_SIZE of both passes, copy-calibrated)",
                           "algorithmic_bytes_per_product": int(alg),
                           "layout_bytes_per_product": int(2 * alg),
                           "layout_GBps": round(2 * alg / sec / 1e9, 2)},
              "lanczos": {"eigenvalues": [float(v) for v in lz["values"]],
                          "residual_estimates": [float(v) for v in lz["resid"]],
                          "steps": lz["iters"], "seconds": round(lanczos_s, 3),
                          "note": "two largest even eigenvalues, residual <= 1e-9 |lambda|, full "
                                  "reorthogonalisation"},
              "ground_state_correlations": {k: round(v, 9) for k, v in corr.items()} | {
                  "seconds": round(corr_s, 5),
                  "note": "Q2, Q4, F of the leading even eigenvector (L_tau -> infinity), "
                          "Walsh-Hadamard transform of its squares on the device"},
              "note": "HIP events around back-to-back products on one stream"}
    if not args.no_cpu_baseline:
        from oracle import transfer
        t0 = time.perf_counter()
        w = transfer.weights(case.L, case.k, case.jx, case.jy)
        tw = time.perf_counter() - t0
        xs = case.vector(0)
        t0 = time.perf_counter()
        transfer.apply(case.L, case.k, case.k_perp, case.jx, case.jy, 1, xs, w)
        ta = time.perf_counter() - t0
        result["cpu_baseline"] = {"value": round(ta * 1e6, 1), "unit": "us per product",
                                  "cores": 1, "kind": "oracle",
                                  "sample": "one even-sector product of the same slice "
                                            f"(numpy, weights precomputed in {tw:.1f} s)",
                                  "host_cpu": host_cpu()}
    print(json.dumps(result), flush=True)


def philox_ceiling(threads: int = 1 << 20, blocks: int = 2048, reps: int = 3):
    """Philox4x32-10 blocks per second of the whole GPU with nothing else in
    the way (the library's probe kernel: the colour pass's counter shape, one
    per-thread word), best of `reps` launches timed with events on their
    stream."""
    import torch
    from paper_2402_03920_amd import qsg
    out = torch.empty(threads, dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    qsg.philox_probe(out, threads, 64, 1, s)  # warm-up
    best = float("inf")
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(s)
        qsg.philox_probe(out, threads, blocks, 1, s)
        b.record(s)
        s.synchronize()
        best = min(best, a.elapsed_time(b) / 1e3)
    return {"blocks_per_s": threads * blocks / best,
            "probe": f"{threads} threads x {blocks} blocks, best of {reps}"}


def summarize(wl, ens):
    """Per slot of the first group shape: mean space and time bond energy per
    site (-Bsp/V, -Bt/V) and <q^2> of the replica-pair overlap, averaged over
    the PT steps of the run and over samples of that shape (from the
    library's integer sums)."""
    import numpy as np
    sums = ens.sums()
    _, p = ens.counters()
    g0 = wl.groups[0]
    same = [i for i, g in enumerate(wl.groups)
            if (g.L, g.L_tau, len(g.gammas)) == (g0.L, g0.L_tau, len(g0.gammas))]
    if p == 0 or not same:
        return {}
    V = g0.L * g0.L * g0.L_tau
    acc = np.zeros((len(g0.gammas), 192))
    for i in same:
        acc += sums[i]
    acc /= len(same) * p
    e_sp = -acc[:, 0:64].mean(axis=1) / V
    e_t = -acc[:, 64:128].mean(axis=1) / V
    q2 = acc[:, 160:192].mean(axis=1) / (V * V)
    return {"shape": f"L={g0.L} L_tau={g0.L_tau} N_Gamma={len(g0.gammas)}",
            "samples": len(same), "pt_steps": p,
            "ladder": getattr(g0, "ladder", "gamma"),
            "ladder_values": [round(float(x), 6) for x in g0.gammas],
            "space_energy_per_site": [round(float(x), 6) for x in e_sp],
            "time_energy_per_site": [round(float(x), 6) for x in e_t],
            "q2": [round(float(x), 6) for x in q2]}


def describe(wl, name):
    if name == "plain-large":
        return (f"{len(wl.groups)} samples x 64 replicas, L=16, L_tau=128, beta=8, "
                f"32 Gammas geometric in [2,4], PT every {wl.pt_every} sweeps")
    if name == "plain-small":
        return "1 sample x 64 replicas, L=8, L_tau=32, beta=4, 16 Gammas in [1.5,4.5]"
    if name == "k-ladder":
        return (f"{len(wl.groups)} samples x 64 replicas, L=16, L_tau=128, one coupling k on "
                f"every bond, 32 k in [0.25,0.33], PT over k every {wl.pt_every} sweeps")
    if name == "uneven":
        return ("256 uneven samples x 64 replicas, L in {8..24}, L_tau in {64,128,256}, "
                "beta=L_tau/16, 24-48 Gammas in [2,4]")
    return "2 groups x 64 samples, L=24, L_tau=2048, beta=128, 48 Gammas in [2.8,3.6]"


def cpu_baseline(wl, n_sweeps):
    """The oracle, as it is, on a bounded sample: one sample of the workload
    for a few sweeps with the OpenMP slot split over the host's cores."""
    from oracle import chain
    cores = len(os.sched_getaffinity(0))
    threads = min(cores, 32)
    g = wl.groups[0]
    if n_sweeps <= 0:  # about 15 s at ~1.4 ns per spin-update on 16 cores
        n_sweeps = max(1, int(round(1.1e10 / g.spin_updates_per_sweep)))
    og = chain.OracleGroup.from_workload_group(g, log_cap=8)
    print(f"[bench] cpu baseline: oracle, 1 sample, {n_sweeps} sweeps, {threads} threads",
          file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    og.run(n_sweeps, 0, threads=threads)
    dt = time.perf_counter() - t0
    upd = n_sweeps * g.spin_updates_per_sweep
    # the same oracle on one core: the first slot of the sample on its own
    # (slots evolve independently between PT steps), about 5-15 s of work
    per_slot = g.spin_updates_per_sweep // len(g.gammas)
    n1 = max(1, int(round(2.5e8 / per_slot)))
    og1 = chain.OracleGroup.single_slot(g, 0, log_cap=8)
    t1 = time.perf_counter()
    og1.run(n1, 0, threads=1)
    dt1 = time.perf_counter() - t1
    upd1 = n1 * per_slot
    return {"value": round(dt / upd * 1e12, 2), "unit": "ps/spin-update", "cores": threads,
            "kind": "oracle",
            "sample": f"1 of {len(wl.groups)} groups (L={g.L}, L_tau={g.L_tau}, "
                      f"{len(g.gammas)} Gammas), {n_sweeps} sweeps, no PT; {upd:.3e} "
                      f"spin-updates in {dt:.1f} s",
            "single_core_ps_per_spin_update": round(dt1 / upd1 * 1e12, 2),
            "single_core_sample": f"slot 0 of the same sample, {n1} sweeps, {upd1:.3e} "
                                  f"spin-updates in {dt1:.1f} s",
            "host_cpu": host_cpu(), "host_cpus_visible": cores}


def host_cpu() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    main()
