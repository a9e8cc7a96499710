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
