"""Per-shape schedule tuning of the colour pass.

A group's colour-pass schedule has two knobs, neither of which changes any
result (the random numbers and decisions do not depend on them; tests check
that every candidate gives the same trajectory):

* `sweep_split`: how many Philox blocks every word goes through before the
  words whose 64 lanes are not all decided are packed into the first waves
  of the block.  Small values pack early (more words travel through LDS),
  large values leave more waves running the long tail of levels; the best
  value depends on the class mix, hence on beta and the ladder.
* `tau_tile`: how many tau planes one thread walks along its column (it
  updates tau_tile/2 words).  Deep walks save loads and index work per word
  but give fewer threads; small slots want shallow walks to fill the chip.

Groups are tuned by class: (L, L_tau, beta, ladder kind and end points);
the number of ladder points only scales the work.  For each class the tuner
builds a sub-ensemble of up to `max_groups` of its groups and times every
candidate's batched colour passes (HIP events on the library's stream, the
median of `repeats` runs of `sweeps` sweeps).  The fastest candidate wins
unless the default is within `tie` of it, which keeps picks stable from run
to run.  Whether a PT chunk runs as one launch per pass or as one fused
launch is the other, ensemble-wide choice (bench.py times both forms).
"""
from __future__ import annotations

import json
import os
from typing import Dict, Iterable, List, Tuple

from . import qsg

SPLITS = (3, 4, 5, 6)
TILES = (2, 4, 8, 16, 32)
DEFAULT = (4, 8)
DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "schedules.json")


def shape_key(g) -> str:
    if getattr(g, "ladder", "gamma") == "k":
        return f"L{g.L}_Lt{g.L_tau}_K{float(g.gammas[0]):.6g}-{float(g.gammas[-1]):.6g}"
    return (f"L{g.L}_Lt{g.L_tau}_b{float(g.beta):.6g}_"
            f"G{float(g.gammas[0]):.6g}-{float(g.gammas[-1]):.6g}")


def valid_tiles(L_tau: int, tiles: Iterable[int] = TILES) -> List[int]:
    """Walk depths that are a distinct power of two dividing L_tau (the
    library takes the largest power of two <= the request dividing L_tau)."""
    return [t for t in tiles if L_tau % t == 0]


def load_cache(path: str = DEFAULT_CACHE) -> Dict[str, Tuple[int, int]]:
    if os.path.exists(path):
        with open(path) as f:
            return {k: tuple(int(x) for x in v) for k, v in json.load(f).items()}
    return {}


def save_cache(cache: Dict[str, Tuple[int, int]], path: str = DEFAULT_CACHE) -> None:
    with open(path + ".tmp", "w") as f:
        json.dump({k: list(v) for k, v in cache.items()}, f, indent=1, sort_keys=True)
    os.replace(path + ".tmp", path)


def _median(xs):
    xs = sorted(xs)
    return xs[len(xs) // 2]


def time_candidates(groups, candidates, sweeps: int = 4, repeats: int = 5, warm: int = 2):
    """Median seconds per sweep of the batched colour passes (no PT) of
    these groups for every (sweep_split, tau_tile) candidate, all in one
    context (the candidates are set with qsg_set_colour_schedule)."""
    import torch
    out = {}
    with qsg.Ensemble(groups, pt_every=0, swaplog_cap=1) as ens:
        ens.init_spins()
        ens.sweep(warm, qsg.QSG_BATCHED)
        for cand in candidates:
            for i in range(len(groups)):
                ens.set_schedule(i, cand[0], cand[1])
            ens.sweep(1, qsg.QSG_BATCHED)
            times = []
            for _ in range(repeats):
                torch.cuda.synchronize()
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record(ens.stream)
                ens.sweep(sweeps, qsg.QSG_BATCHED | qsg.QSG_NO_PT)
                b.record(ens.stream)
                torch.cuda.synchronize()
                times.append(a.elapsed_time(b) / 1e3 / sweeps)
            out[cand] = _median(times)
    return out


def tune(groups, splits: Iterable[int] = SPLITS, tiles: Iterable[int] = TILES,
         cache: Dict[str, Tuple[int, int]] | None = None, max_groups: int = 16,
         tie: float = 0.01, log=None) -> Dict[str, Tuple[int, int]]:
    """Best (sweep_split, tau_tile) for every class present in `groups`."""
    cache = {} if cache is None else cache
    by_class: Dict[str, List] = {}
    for g in groups:
        by_class.setdefault(shape_key(g), []).append(g)
    for key, gs in by_class.items():
        if key in cache:
            continue
        cands = [(s, t) for s in splits for t in valid_tiles(gs[0].L_tau, tiles)]
        default = (DEFAULT[0], max(t for t in valid_tiles(gs[0].L_tau) if t <= DEFAULT[1]))
        if default not in cands:
            cands.append(default)
        times = time_candidates(gs[:max_groups], cands)
        best = min(times, key=times.get)
        if times[default] <= times[best] * (1.0 + tie):
            best = default
        cache[key] = best
        if log:
            log(f"[autotune] {key}: " + ", ".join(f"{c[0]}/{c[1]}:{t * 1e6:.1f}us"
                                                  for c, t in sorted(times.items()))
                + f" -> split {best[0]}, tile {best[1]}")
    return cache


def apply(ens, cache: Dict[str, Tuple[int, int]]) -> int:
    """Set every group's schedule from the cache; returns how many were set."""
    n = 0
    for i, g in enumerate(ens.groups):
        k = shape_key(g)
        if k in cache:
            split, tile = cache[k]
            ens.set_schedule(i, split, tile)
            n += 1
    return n
