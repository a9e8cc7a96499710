"""Helpers shared by the GPU parity tests: run the HIP path and the oracle
on the same seeded groups and compare everything bit for bit."""
import numpy as np

from oracle import chain


def oracle_groups(groups, log_cap):
    return [chain.OracleGroup.from_workload_group(g, log_cap=log_cap) for g in groups]


def compare_state(ens, ogs, check_sums=True, groups=None):
    """Assert that the GPU ensemble and the oracle groups hold identical
    states; oracle group i is the ensemble's group groups[i] (default i).
    Returns the number of words compared."""
    words = 0
    energies = ens.energies()
    walkers = ens.walkers()
    accepts = ens.accepts()
    rts = ens.roundtrips()
    logs = ens.swaplog_rows()
    sums = ens.sums() if check_sums else None
    hists = ens.histograms() if check_sums else None
    t, p = ens.counters()
    for j, og in enumerate(ogs):
        i = groups[j] if groups is not None else j
        assert (t, p) == (og.t, og.p), (i, t, p, og.t, og.p)
        sp = ens.get_spins(i)
        if not np.array_equal(sp, og.spins):
            bad = np.nonzero(sp != og.spins)[0]
            raise AssertionError(f"group {i}: {bad.size} spin words differ, first at {bad[:8]}")
        words += sp.size
        N = og.N
        e = energies[i]
        assert np.array_equal(e[:, :, 0], og.Bsp.reshape(N, 64)), f"group {i}: Bsp"
        assert np.array_equal(e[:, :, 1], og.Bt.reshape(N, 64)), f"group {i}: Bt"
        assert np.array_equal(walkers[i], og.walker.reshape(N, 64)), f"group {i}: walkers"
        if N > 1:
            assert np.array_equal(accepts[i], og.acc[:N - 1]), f"group {i}: accept counts"
            assert np.array_equal(logs[i], og.swaplog_rows()), f"group {i}: swap log"
        rt = rts[i]
        assert np.array_equal(rt["state"], og.rt_state.reshape(N, 64)), f"group {i}: rt state"
        assert np.array_equal(rt["count"], og.rt_count.reshape(N, 64)), f"group {i}: rt count"
        assert np.array_equal(rt["sum"], og.rt_sum.reshape(N, 64)), f"group {i}: rt sum"
        assert np.array_equal(rt["t_last"], og.rt_tlast.reshape(N, 64)), f"group {i}: rt t_last"
        if check_sums:
            s = sums[i]
            assert np.array_equal(s[:, 0:64], og.sum_Bsp.reshape(N, 64)), f"group {i}: sum Bsp"
            assert np.array_equal(s[:, 64:128], og.sum_Bt.reshape(N, 64)), f"group {i}: sum Bt"
            assert np.array_equal(s[:, 128:160], og.sum_q.reshape(N, 32)), f"group {i}: sum q"
            assert np.array_equal(s[:, 160:192], og.sum_q2.reshape(N, 32)), f"group {i}: sum q2"
            assert np.array_equal(hists[i], og.hist.reshape(N, 1024)), f"group {i}: Bt histogram"
    return words


# ---------------------------------------------------------------------------
# Digests of a group's full state, for workloads whose oracle run takes
# minutes: tests/golden/make_oracle_records.py stores the oracle's record and
# the GPU tests compare their own record with it field by field.  Arrays are
# hashed in a fixed dtype and order, so equal digests mean equal arrays.

def _digest(a, dtype="<i8"):
    import hashlib
    return hashlib.sha256(np.ascontiguousarray(np.asarray(a), dtype=dtype).tobytes()).hexdigest()


def state_record(t, p, N, V, spins, Bsp, Bt, walker, acc, swaplog, rt, sums, hist):
    """Record of one group: spins per slot [N*V], Bsp/Bt/walker [N][64],
    acc [N-1], swaplog rows oldest first [p][N-1], round-trip fields
    (state, count, sum, t_last) [N][64], sums [N][192], hist [N][1024]."""
    rec = {"t": int(t), "p": int(p),
           "spins": [_digest(spins[g * V:(g + 1) * V], "<u8") for g in range(N)],
           "Bsp": _digest(Bsp), "Bt": _digest(Bt), "walker": _digest(walker),
           "rt": {k: _digest(rt[k]) for k in ("state", "count", "sum", "t_last")},
           "sums": _digest(sums), "hist": _digest(hist)}
    if N > 1:
        rec["acc"] = [int(x) for x in np.asarray(acc).reshape(-1)]
        rec["swaplog"] = [[int(x) for x in row] for row in np.asarray(swaplog, dtype=np.uint64)]
    return rec


def oracle_record(og):
    N, V = og.N, og.V
    sums = np.concatenate([og.sum_Bsp.reshape(N, 64), og.sum_Bt.reshape(N, 64),
                           og.sum_q.reshape(N, 32), og.sum_q2.reshape(N, 32)], axis=1)
    rt = {"state": og.rt_state.reshape(N, 64), "count": og.rt_count.reshape(N, 64),
          "sum": og.rt_sum.reshape(N, 64), "t_last": og.rt_tlast.reshape(N, 64)}
    return state_record(og.t, og.p, N, V, og.spins, og.Bsp.reshape(N, 64), og.Bt.reshape(N, 64),
                        og.walker.reshape(N, 64), og.acc[:max(N - 1, 1)], og.swaplog_rows(), rt,
                        sums, og.hist.reshape(N, 1024))


def gpu_record(ens, i, cache=None):
    """The same record from the GPU ensemble's group i (cache: dict holding
    the ensemble-wide measurements, filled on first use)."""
    c = cache if cache is not None else {}
    if not c:
        c.update(energies=ens.energies(), walkers=ens.walkers(), accepts=ens.accepts(),
                 rts=ens.roundtrips(), logs=ens.swaplog_rows(), sums=ens.sums(),
                 hists=ens.histograms(), counters=ens.counters())
    t, p = c["counters"]
    e = c["energies"][i]
    N = e.shape[0]
    spins = ens.get_spins(i)
    V = spins.size // N
    return state_record(t, p, N, V, spins, e[:, :, 0], e[:, :, 1], c["walkers"][i],
                        c["accepts"][i], c["logs"][i], c["rts"][i], c["sums"][i], c["hists"][i])


STATE_KEYS = ("t", "p", "spins", "Bsp", "Bt", "walker", "rt", "sums", "hist", "acc", "swaplog")


def compare_records(got, want, name):
    """Assert the state fields of two records are equal (the stored record
    also carries the case's description), naming the first that differs."""
    assert all(k in want for k in STATE_KEYS[:9]), f"{name}: stored record incomplete"
    for key in (k for k in STATE_KEYS if k in want):
        if key == "spins":
            bad = [g for g, (a, b) in enumerate(zip(got["spins"], want["spins"])) if a != b]
            assert not bad and len(got["spins"]) == len(want["spins"]), \
                f"{name}: spins of slots {bad[:8]} differ"
        else:
            assert got.get(key) == want[key], f"{name}: {key} differs"
