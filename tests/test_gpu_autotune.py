"""The colour-pass tuner on the GPU: its picks are stable from run to run,
and a tuned ensemble follows the same trajectory as an untuned one.

Stability is judged by time, not by identity: two candidates within the
tuner's tie margin are equally good, so the second run must time the first
run's pick within a few per cent of its own best.  The walk depth is one
for the whole ensemble, the split one per class.
"""
import sys

import numpy as np
import pytest

import qsg_workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU-only hosts, never run there
    pytest.skip("no GPU", allow_module_level=True)

from paper_2402_03920_amd import autotune, qsg  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _two_class_groups():
    """16 samples of the large plain shape (L=16, L_tau=128, 32 Gammas) and
    16 of a deeper, smaller one (L=12, L_tau=256): two classes."""
    big = W.plain_large(n_samples=16).groups
    small = [W.Group(12, 256, 16.0, W.geometric_ladder(2.0, 4.0, 24), 100 + i, W.MC_SEED,
                     W._replicas(500 + i)) for i in range(16)]
    return big + small


def test_tuner_picks_are_stable_across_two_runs():
    torch.cuda.set_device(0)
    groups = _two_class_groups()
    runs = []
    for r in range(2):
        rep = {}
        autotune.tune(groups, report=rep, log=say)
        runs.append(rep)
    first, second = runs
    classes = [k for k in first if k != "tiles"]
    assert sorted(classes) == sorted(k for k in second if k != "tiles") and len(classes) == 2
    # one walk depth for the ensemble: the first run's, timed in the second
    # run, is as good as the second run's
    d1, d2 = first[classes[0]]["pick"][1], second[classes[0]]["pick"][1]
    say(f"walk depth: run 1 {d1}, run 2 {d2}")
    assert all(first[k]["pick"][1] == d1 and second[k]["pick"][1] == d2 for k in classes)
    assert second["tiles"][d1] <= second["tiles"][d2] * 1.05, (d1, d2, second["tiles"])
    for key in classes:
        s1, s2 = first[key]["pick"][0], second[key]["pick"][0]
        say(f"{key}: split run 1 {s1}, run 2 {s2}")
        if s1 == s2 or d1 != d2:
            continue
        t2 = {c[0]: t for c, t in second[key]["splits"].items()}
        assert t2[s1] <= t2[s2] * 1.05, (key, s1, s2, t2)


def test_tuned_ensemble_follows_the_untuned_trajectory():
    torch.cuda.set_device(0)
    groups = _two_class_groups()[::4]
    cache = autotune.tune(groups, splits=(3, 6), tiles=(2, 32), scale_words=1 << 22)
    assert len(cache) == 2
    # a schedule other than the default on some class, so the check means something
    cache = {k: ((6, 2) if i == 0 else (3, 32)) for i, k in enumerate(sorted(cache))}
    out = []
    for tuned in (False, True):
        with qsg.Ensemble(groups, pt_every=5, swaplog_cap=16) as ens:
            if tuned:
                assert autotune.apply(ens, cache) == len(groups)
            ens.init_spins()
            name, flags, _ = autotune.pick_form(ens, chunks=1, repeats=1)
            ens.sweep(10, flags)
            out.append([ens.get_spins(i) for i in range(len(groups))] + list(ens.energies()))
    assert len(out[0]) == len(out[1]) == 2 * len(groups)
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)
