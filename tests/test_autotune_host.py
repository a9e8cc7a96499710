"""Host logic of the colour-pass tuner (no GPU): how a class is scaled to
the ensemble's size, the tie rule that keeps the default, and the schedule
cache's round trip."""
import numpy as np

import qsg_workloads as W
from paper_2402_03920_amd import autotune


def test_at_scale_repeats_the_class_until_it_holds_the_words():
    gs = W.uneven_ensemble(32).groups[:3]
    words = [autotune.group_words(g) for g in gs]
    assert words == [g.words for g in gs]
    # every group at least once, in order, even when they already exceed the target
    assert autotune.at_scale(gs, 1) == gs
    target = 5 * sum(words) + 1
    out = autotune.at_scale(gs, target)
    assert sum(autotune.group_words(g) for g in out) >= target
    assert sum(autotune.group_words(g) for g in out[:-1]) < target
    assert all(out[i] is gs[i % 3] for i in range(len(out)))


def test_shape_key_ignores_the_number_of_ladder_points_only():
    a = W.Group(12, 64, 4.0, W.geometric_ladder(2.0, 4.0, 24), 0, W.MC_SEED, W._replicas(1))
    b = W.Group(12, 64, 4.0, W.geometric_ladder(2.0, 4.0, 40), 7, W.MC_SEED, W._replicas(9))
    c = W.Group(12, 64, 4.5, W.geometric_ladder(2.0, 4.0, 24), 0, W.MC_SEED, W._replicas(1))
    d = W.Group(12, 128, 4.0, W.geometric_ladder(2.0, 4.0, 24), 0, W.MC_SEED, W._replicas(1))
    assert autotune.shape_key(a) == autotune.shape_key(b)
    assert len({autotune.shape_key(g) for g in (a, c, d)}) == 3


def test_the_default_wins_ties_within_the_margin():
    t = {(4, 8): 1.000, (4, 16): 0.995, (3, 8): 1.2}
    assert autotune._pick(t, (4, 8), 0.01) == (4, 8)
    t[(4, 16)] = 0.98
    assert autotune._pick(t, (4, 8), 0.01) == (4, 16)


def test_schedule_cache_round_trip(tmp_path):
    cache = {"L8_Lt64_b4_G2-4": (4, 16), "L16_Lt128_K0.33-0.25": (5, 8)}
    path = str(tmp_path / "s.json")
    autotune.save_cache(cache, path)
    assert autotune.load_cache(path) == cache
    assert autotune.load_cache(str(tmp_path / "missing.json")) == {}
