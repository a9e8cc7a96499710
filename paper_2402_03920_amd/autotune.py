"""Per-shape schedule tuning of the colour pass, and the choice of launch form.

A group's colour-pass schedule has two knobs, neither of which changes any
result (the random numbers and decisions do not depend on them; tests check
that every candidate gives the same trajectory):

* `tau_tile`: how many tau planes one thread walks along its column (it
  updates tau_tile/2 words).  Deep walks save loads and index work per word
  but give fewer threads; small ensembles want shallow walks to fill the
  chip.
* `sweep_split`: how many Philox blocks every word goes through before the
  words whose 64 lanes are not all decided are packed into the first waves
  of the block.  Small values pack early (more words travel through LDS),
  large values leave more waves running the long tail of levels; the best
  value depends on the class mix, hence on beta and the ladder.

The walk depth is chosen for the whole ensemble: the batched launch deals
its blocks to the eight XCDs in equal contiguous runs, so blocks of unequal
depth (unequal work) leave some XCDs idle at the end of the pass; a mix of
per-class depths measured 12 % slower than one depth for all.  The tuner
times the whole ensemble under every depth (the library takes, per group,
the largest power of two not above the request that divides L_tau).  The
split is chosen per class (L, L_tau, beta, ladder kind and end points; the
number of ladder points only scales the work), at that depth.  Both are
timed at the size of the whole ensemble, up to SCALE_WORDS: the groups are
repeated until the timed ensemble holds that many words (a class timed on
its own would favour shallow walks that lose once the other classes share
the chip; beyond 2^26 words every candidate fills the chip several times
over).  Each timing is the median of `repeats` runs of `sweeps` sweeps (HIP
events on the library's stream); a candidate replaces the default only
when it is faster by more than `tie`, which keeps picks stable from run to
run.

`pick_form` makes the other, ensemble-wide choice: whether a PT chunk runs
as one launch per colour pass or as one fused launch for all its sweeps.
`pick_plain_tile` chooses the depth of per-sample launches, which fill the
chip one group at a time.
"""
from __future__ import annotations

import json
import os
from typing import Dict, Iterable, List, Tuple

from . import qsg

SPLITS = (3, 4, 5, 6)
TILES = (2, 4, 8, 16, 32)
DEFAULT = (4, 8)
SCALE_WORDS = 1 << 26
DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "schedules.json")


def shape_key(g) -> str:
    if getattr(g, "ladder", "gamma") == "k":
        return f"L{g.L}_Lt{g.L_tau}_K{float(g.gammas[0]):.6g}-{float(g.gammas[-1]):.6g}"
    return (f"L{g.L}_Lt{g.L_tau}_b{float(g.beta):.6g}_"
            f"G{float(g.gammas[0]):.6g}-{float(g.gammas[-1]):.6g}")


def group_words(g) -> int:
    return len(g.gammas) * g.L * g.L * g.L_tau


def at_scale(gs: List, words: int) -> List:
    """The class's groups, repeated in order until they hold at least
    `words` words (at least every group once)."""
    out, have, i = [], 0, 0
    while i < len(gs) or have < words:
        g = gs[i % len(gs)]
        out.append(g)
        have += group_words(g)
        i += 1
    return out


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


def _timer(stream):
    import torch

    def timed(fn):
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / 1e3
    return timed


def time_candidates(ens, candidates, sweeps: int = 4, repeats: int = 5):
    """Median seconds per sweep of the ensemble's batched colour passes (no
    PT) for every (sweep_split, tau_tile) candidate, set on every group with
    qsg_set_colour_schedule."""
    timed = _timer(ens.stream)
    out = {}
    for cand in candidates:
        for i in range(ens.n):
            ens.set_schedule(i, cand[0], cand[1])
        ens.sweep(1, qsg.QSG_BATCHED | qsg.QSG_NO_PT)
        out[cand] = _median([timed(lambda: ens.sweep(sweeps, qsg.QSG_BATCHED | qsg.QSG_NO_PT))
                             / sweeps for _ in range(repeats)])
    return out


def _pick(times, default, tie):
    best = min(times, key=times.get)
    return default if times[default] <= times[best] * (1.0 + tie) else best


def tune(groups, splits: Iterable[int] = SPLITS, tiles: Iterable[int] = TILES,
         cache: Dict[str, Tuple[int, int]] | None = None, tie: float = 0.01,
         scale_words: int | None = None, log=None, report: Dict | None = None
         ) -> Dict[str, Tuple[int, int]]:
    """(sweep_split, tau_tile) for every class present in `groups`: one walk
    depth for the ensemble, a split per class, timed at `scale_words` words
    (default: the whole ensemble's, at most SCALE_WORDS).  Classes already
    in `cache` keep their entry; the others get the depth tuned now.
    `report`, if given, receives the timings: report["tiles"] per depth and
    report[class] = {"splits": ..., "pick": ...}."""
    cache = {} if cache is None else cache
    by_class: Dict[str, List] = {}
    for g in groups:
        by_class.setdefault(shape_key(g), []).append(g)
    todo = [k for k in by_class if k not in cache]
    if not todo:
        return cache
    words = min(sum(group_words(g) for g in groups), SCALE_WORDS) if scale_words is None \
        else scale_words
    split0, tile0 = DEFAULT
    with qsg.Ensemble(at_scale(list(groups), words), pt_every=0, swaplog_cap=1) as ens:
        ens.init_spins()
        ens.sweep(2, qsg.QSG_BATCHED | qsg.QSG_NO_PT)
        t_tiles = time_candidates(ens, [(split0, t) for t in sorted(set(tiles) | {tile0})])
    tile = _pick(t_tiles, (split0, tile0), tie)[1]
    if report is not None:
        report["tiles"] = {c[1]: t for c, t in t_tiles.items()}
    if log:
        log(f"[autotune] walk depth at {words} words: "
            + ", ".join(f"{c[1]}:{t * 1e6:.1f}us" for c, t in sorted(t_tiles.items()))
            + f" -> tile {tile}")
    for key in todo:
        gs = by_class[key]
        with qsg.Ensemble(at_scale(gs, words), pt_every=0, swaplog_cap=1) as ens:
            ens.init_spins()
            ens.sweep(2, qsg.QSG_BATCHED | qsg.QSG_NO_PT)
            t_splits = time_candidates(ens, [(s, tile) for s in sorted(set(splits) | {split0})])
        best = _pick(t_splits, (split0, tile), tie)
        cache[key] = best
        if report is not None:
            report[key] = {"splits": t_splits, "pick": best}
        if log:
            log(f"[autotune] {key} at {words} words: "
                + ", ".join(f"{c[0]}:{t * 1e6:.1f}us" for c, t in sorted(t_splits.items()))
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


def pick_plain_tile(ens, cache: Dict[str, Tuple[int, int]], tiles: Iterable[int] = TILES,
                    sweeps: int = 2, repeats: int = 3):
    """Walk depth for per-sample launches (QSG_PLAIN), which fill the chip
    one group at a time and so want shallower walks than the batched pass:
    every depth is timed over the whole ensemble (each group keeps its
    cached split).  Leaves the ensemble on the best depth; returns it and
    the seconds per sweep of every depth."""
    timed = _timer(ens.stream)
    times = {}
    for tile in sorted(set(tiles)):
        for i, g in enumerate(ens.groups):
            ens.set_schedule(i, cache.get(shape_key(g), DEFAULT)[0], tile)
        ens.sweep(1, qsg.QSG_PLAIN | qsg.QSG_NO_PT)
        times[tile] = _median([timed(lambda: ens.sweep(sweeps, qsg.QSG_PLAIN | qsg.QSG_NO_PT))
                               / sweeps for _ in range(repeats)])
    best = min(times, key=times.get)
    for i, g in enumerate(ens.groups):
        ens.set_schedule(i, cache.get(shape_key(g), DEFAULT)[0], best)
    return best, times


FORMS = {"per-pass": qsg.QSG_BATCHED | qsg.QSG_GRAPH,
         "fused": qsg.QSG_BATCHED | qsg.QSG_GRAPH | qsg.QSG_FUSED}


def pick_form(ens, chunks: int = 2, repeats: int = 3):
    """The faster batched form of a PT chunk for this ensemble, both replayed
    as HIP graphs: one launch per colour pass over every group, or one fused
    launch per chunk (a block per slot).  Returns (name, flags, seconds per
    chunk of each form).  Both forms give the same trajectory; timing them
    advances the ensemble."""
    timed = _timer(ens.stream)
    pe = ens.cfg.pt_every
    times = {}
    for name, fl in FORMS.items():
        ens.sweep(pe, fl)  # capture + warm
        times[name] = _median([timed(lambda: ens.sweep(pe * chunks, fl)) / chunks
                               for _ in range(repeats)])
    name = min(times, key=times.get)
    return name, FORMS[name], times
