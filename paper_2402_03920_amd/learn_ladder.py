"""Train the ladder MLP on acceptance measured in plain runs, then compare
learned and geometric ladders on fresh samples.

    python -m paper_2402_03920_amd.learn_ladder --out ladder.json

Training data: every group of the small plain workload (one sample), of the
large plain workload (64 samples) and of the uneven ensemble (256 samples)
is run with its geometric ladder; the exchange acceptance of each pair
(second half of the run) gives the target ladder.  Evaluation: fresh
samples with L in {12, 16, 20, 24}, L_tau = 256, beta = 16, 32 Gammas in
[2, 4], each run twice from the same spins and random numbers, once with the
geometric ladder and once with the learned one (the geometric ladder where
the predicted acceptance is below the floor).
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time
from dataclasses import replace

import numpy as np

from . import ladder, qsg


def _features_of(ens, groups) -> np.ndarray:
    X = []
    for i, g in enumerate(groups):
        jx, jy = ens.get_couplings(i)
        ff = ladder.frustrated_fraction(jx, jy, g.L)
        X.append(ladder.features(g.L, g.L_tau, g.beta, ff, g.gammas[0], g.gammas[-1]))
    return np.stack(X)


def _features_of_groups(groups) -> np.ndarray:
    """Features of groups that are not running (couplings built on the GPU
    in a throwaway context)."""
    with qsg.Ensemble(groups, pt_every=10, swaplog_cap=1) as ens:
        return _features_of(ens, groups)


def collect(groups, sweeps: int, pt_every: int = 10, flags=None, log=print):
    """Run groups with their own ladders; return features, targets and the
    acceptance of every pair over the second half of the run."""
    import torch
    if flags is None:
        flags = qsg.QSG_BATCHED | qsg.QSG_GRAPH
    half = (sweeps // 2 // pt_every) * pt_every
    with qsg.Ensemble(groups, pt_every=pt_every, swaplog_cap=8) as ens:
        X = _features_of(ens, groups)
        ens.init_spins()
        ens.sweep(half, flags)
        a0 = ens.accepts()
        p0 = ens.counters()[1]
        ens.sweep(sweeps - half, flags)
        a1 = ens.accepts()
        p1 = ens.counters()[1]
    rates = [(b - a).astype(np.float64) / (64.0 * max(p1 - p0, 1)) for a, b in zip(a0, a1)]
    T, logL = [], []
    for g, r in zip(groups, rates):
        inc, lg = ladder.targets_from_acceptance(g.gammas, r)
        T.append(inc)
        logL.append(lg)
    log(f"[ladder] collected {len(groups)} runs of {sweeps} sweeps")
    return X, np.stack(T), np.array(logL, dtype=np.float32), rates


def compare(model: ladder.LadderMLP, groups, sweeps: int, floor: float = 0.2,
            pt_every: int = 10, log=print):
    """Geometric against learned (with fallback) ladders on the same samples,
    spins and random numbers."""
    import torch
    flags = qsg.QSG_BATCHED | qsg.QSG_GRAPH
    with qsg.Ensemble(groups, pt_every=pt_every, swaplog_cap=8) as ens:
        X = _features_of(ens, groups)
    gmin = np.array([g.gammas[0] for g in groups])
    gmax = np.array([g.gammas[-1] for g in groups])
    pred, acc_pred = model.predict(X, gmin, gmax)
    chosen, used = ladder.choose(pred, acc_pred, gmin, gmax, floor)
    learned_groups = [replace(g, gammas=chosen[i]) for i, g in enumerate(groups)]
    out = {}
    for name, gs in (("geometric", groups), ("learned", learned_groups)):
        st = ladder.run_and_measure(gs, sweeps, pt_every, flags)
        acc = np.stack([a for a in st.acc_rate])
        out[name] = {
            "round_trips": int(st.rt_count.sum()),
            "round_trips_per_hour": float(st.rt_count.sum() / (st.wall_s / 3600.0)),
            "mean_round_trip_pt_steps": float(np.nansum(st.rt_time * st.rt_count) /
                                              max(st.rt_count.sum(), 1)),
            "rt_per_sample": st.rt_count.tolist(),
            "acceptance_min": float(acc.min()),
            "acceptance_mean": float(acc.mean()),
            "acceptance_std_within_sample_mean": float(acc.std(axis=1).mean()),
            "acceptance_min_per_sample": acc.min(axis=1).tolist(),
            "wall_s": st.wall_s,
            "pt_steps": st.pt_steps,
        }
        log(f"[ladder] {name}: {out[name]['round_trips']} round trips, "
            f"acceptance min {out[name]['acceptance_min']:.3f} mean {out[name]['acceptance_mean']:.3f}")
    rg = np.array(out["geometric"]["rt_per_sample"], dtype=float)
    rl = np.array(out["learned"]["rt_per_sample"], dtype=float)
    d = rl - rg
    out["paired_round_trip_gain"] = {
        "mean": float(d.mean()), "stderr": float(d.std(ddof=1) / math.sqrt(len(d))) if len(d) > 1 else 0.0,
        "mean_learned_only": float(d[used].mean()) if used.any() else 0.0,
    }
    out["fallback_fraction"] = float(1.0 - used.mean())
    out["predicted_acceptance"] = acc_pred.tolist()
    out["L"] = [g.L for g in groups]
    return out


def main(argv=None):
    import qsg_workloads as W
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--train-sweeps", type=int, default=2000)
    ap.add_argument("--eval-sweeps", type=int, default=10000)
    ap.add_argument("--eval-samples", type=int, default=128)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--uneven-samples", type=int, default=256)
    ap.add_argument("--focus-sweeps", type=int, default=50000,
                    help="second, longer comparison on the samples whose learned ladder "
                         "passed the floor (0: skip)")
    ap.add_argument("--out", default="")
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    t0 = time.time()
    sets = [W.plain_small().groups, W.plain_large().groups,
            W.uneven_ensemble(args.uneven_samples).groups]
    Xs, Ts, Ls = [], [], []
    for gs in sets:
        X, T, L, _ = collect(gs, args.train_sweeps, log=log)
        Xs.append(X)
        Ts.append(T)
        Ls.append(L)
    X, T, L = np.concatenate(Xs), np.concatenate(Ts), np.concatenate(Ls)
    model = ladder.LadderMLP(seed=0, bf16=True)
    hist = model.fit(X, T, L, steps=args.steps, lr=args.lr, log_every=max(args.steps // 10, 1))
    log(f"[ladder] trained on {len(X)} runs: loss {hist[0]:.4f} -> {hist[-1]:.4f}")
    ev = W.ladder_eval(n_samples=args.eval_samples).groups
    res = compare(model, ev, args.eval_sweeps, log=log)
    if args.focus_sweeps:
        keep = [g for g, a in zip(ev, res["predicted_acceptance"]) if a >= 0.2]
        if keep:
            log(f"[ladder] focused comparison: {len(keep)} samples, {args.focus_sweeps} sweeps")
            res["focused"] = compare(model, keep, args.focus_sweeps, log=log)
    res["train"] = {"runs": int(len(X)), "loss_history": hist, "steps": args.steps,
                    "train_sweeps": args.train_sweeps}
    res["elapsed_s"] = time.time() - t0
    js = json.dumps(res)
    if args.out:
        with open(args.out, "w") as f:
            f.write(js)
    print(json.dumps({k: v for k, v in res.items()
                      if k in ("paired_round_trip_gain", "fallback_fraction")}))
    for key in ("geometric", "learned"):
        print(key, {k: res[key][k] for k in ("round_trips", "round_trips_per_hour",
                                              "mean_round_trip_pt_steps", "acceptance_min",
                                              "acceptance_mean")})
    if "focused" in res:
        f = res["focused"]
        print("focused", f["paired_round_trip_gain"],
              {k: (f["geometric"][k], f["learned"][k]) for k in
               ("round_trips", "round_trips_per_hour", "mean_round_trip_pt_steps",
                "acceptance_min", "acceptance_std_within_sample_mean")})


if __name__ == "__main__":
    main()
