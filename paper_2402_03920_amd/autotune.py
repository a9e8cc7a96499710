"""Per-shape schedule tuning of the colour pass.

The schedule of a group is `sweep_split`: how many Philox blocks every word
of a colour pass goes through before the words whose 64 lanes are not all
decided are packed into the first waves of the block.  Small values pack
early (more words travel through LDS), large values leave more waves
running the long tail of levels.  The best value depends on the class mix,
hence on (L, L_tau, beta, ladder), so the tuner times candidates on the GPU
for each shape of an ensemble and caches the winner in a JSON file.

Every candidate computes exactly the same trajectory (the random numbers
and decisions do not depend on the schedule); tests check that.
"""
from __future__ import annotations

import json
import os
from typing import Dict, Iterable, List

from . import qsg

CANDIDATES = (2, 3, 4, 5, 6, 16)
DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "schedules.json")


def shape_key(g) -> str:
    if getattr(g, "ladder", "gamma") == "k":
        return (f"L{g.L}_Lt{g.L_tau}_N{len(g.gammas)}_"
                f"K{float(g.gammas[0]):.6g}-{float(g.gammas[-1]):.6g}")
    return (f"L{g.L}_Lt{g.L_tau}_N{len(g.gammas)}_b{float(g.beta):.6g}_"
            f"G{float(g.gammas[0]):.6g}-{float(g.gammas[-1]):.6g}")


def load_cache(path: str = DEFAULT_CACHE) -> Dict[str, int]:
    if os.path.exists(path):
        with open(path) as f:
            return {k: int(v) for k, v in json.load(f).items()}
    return {}


def save_cache(cache: Dict[str, int], path: str = DEFAULT_CACHE) -> None:
    with open(path + ".tmp", "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(path + ".tmp", path)


def time_schedule(groups, split: int, sweeps: int = 4, warm: int = 2) -> float:
    """Seconds per sweep of the batched colour passes with one schedule for
    every group (no PT), from random spins after `warm` sweeps."""
    import torch
    with qsg.Ensemble(groups, pt_every=0, swaplog_cap=1, sweep_split=split) as ens:
        ens.init_spins()
        ens.sweep(warm, qsg.QSG_BATCHED)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(ens.stream)
        ens.sweep(sweeps, qsg.QSG_BATCHED)
        b.record(ens.stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / 1e3 / sweeps


def tune(groups, candidates: Iterable[int] = CANDIDATES, cache: Dict[str, int] | None = None,
         max_groups_per_shape: int = 8, log=None) -> Dict[str, int]:
    """Best schedule for every shape present in `groups` (timed on up to
    `max_groups_per_shape` groups of that shape)."""
    cache = {} if cache is None else cache
    by_shape: Dict[str, List] = {}
    for g in groups:
        by_shape.setdefault(shape_key(g), []).append(g)
    for key, gs in by_shape.items():
        if key in cache:
            continue
        sample = gs[:max_groups_per_shape]
        times = {c: time_schedule(sample, c) for c in candidates}
        best = min(times, key=times.get)
        cache[key] = best
        if log:
            log(f"[autotune] {key}: " + ", ".join(f"{c}:{t * 1e3:.3f}ms" for c, t in times.items())
                + f" -> {best}")
    return cache


def apply(ens, cache: Dict[str, int]) -> int:
    """Set every group's schedule from the cache; returns how many were set."""
    n = 0
    for i, g in enumerate(ens.groups):
        k = shape_key(g)
        if k in cache:
            ens.set_schedule(i, cache[k])
            n += 1
    return n
