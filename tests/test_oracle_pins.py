"""Pins of the oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each check is anchored on a
published known-answer vector, a closed form derived independently (exact
enumeration, transfer matrix, exact stationarity of the update operator),
a limit, or an invariant of the dynamics.
"""
import math

import numpy as np
import pytest

from oracle import chain, exact, tables
import qsg_workloads as W

U32 = 2 ** 32


# --------------------------------------------------------------------------
# Philox4x32-10 (paper Sec. 2.1.1 uses D.E. Shaw's philox_4x32_10)
# --------------------------------------------------------------------------
def test_philox_known_answers(philox_kat):
    for ctr, key, want in philox_kat:
        got = chain.philox(ctr, key)
        assert [int(x) for x in got] == want


def test_metropolis_r_is_uniform_32bit():
    """Lane numbers assembled from bit-sliced levels are uniform 32-bit
    integers: acceptance frequency of r <= thr is (thr+1)/2^32."""
    rs = np.concatenate([chain.metropolis_r(42, 7, s, t, g)
                         for s in range(40) for t in range(5) for g in range(3)])
    n = rs.size
    for thr in (2 ** 31 - 1, 2 ** 30 - 1, 3 * 2 ** 30 - 1, 2 ** 28 - 1):
        p = (thr + 1) / U32
        f = np.mean(rs.astype(np.uint64) <= thr)
        assert abs(f - p) < 5 * math.sqrt(p * (1 - p) / n)
    # every bit position is fair
    for b in range(32):
        f = np.mean((rs >> b) & 1)
        assert abs(f - 0.5) < 5 * math.sqrt(0.25 / n)


# --------------------------------------------------------------------------
# Threshold tables (paper Sec. 1: Gamma(k); App. B: daemon levels e^-4k..)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("k", [0.125, 0.29, 0.32])
def test_equal_coupling_collapse(k):
    """With Gamma = -ln tanh(k)/(2k) (the paper's equal-coupling relation)
    the time coupling equals k, so a flip's weight change depends only on
    the total number of unsatisfied bonds n = n_s + n_t, and the only
    non-trivial factors are the paper's three daemon levels e^-4k, e^-8k,
    e^-12k (App. B)."""
    L_tau = 64
    beta = k * L_tau
    G = tables.gamma_of_equal_coupling(k)
    thr = tables.metropolis_thresholds(beta, L_tau, [G])[0]
    by_total = {}
    for ns in range(5):
        for nt in range(3):
            by_total.setdefault(ns + nt, set()).add(int(thr[ns, nt]))
    for n, vals in by_total.items():
        assert len(vals) == 1, (n, vals)
    for n in range(3, 7):
        assert by_total[n] == {U32 - 1}
    # daemon level probabilities as stated in App. B, from Python's float
    # exp: the threshold over 2^32 matches them to the table's quantum
    for n, m in ((2, 1), (1, 2), (0, 3)):
        (v,) = by_total[n]
        assert abs((v + 1) / U32 - math.exp(-4 * k * m)) < 2.0 / U32


def test_thresholds_monotone_and_saturated():
    beta, L_tau = 8.0, 128
    lad = W.geometric_ladder(2.0, 4.0, 8)
    thr = tables.metropolis_thresholds(beta, L_tau, lad).astype(np.int64)
    k = beta / L_tau
    for g, G in enumerate(lad):
        kp = -0.5 * math.log(math.tanh(beta * G / L_tau))
        pairs = sorted(((4 * k * (2 - ns) + 4 * kp * (1 - nt), thr[g, ns, nt])
                        for ns in range(5) for nt in range(3)))
        # non-increasing threshold in the energy change
        for (e0, t0), (e1, t1) in zip(pairs, pairs[1:]):
            assert t1 <= t0
        for e, t in pairs:
            if e <= 0:
                assert t == U32 - 1
            else:
                assert abs((t + 1) / U32 - math.exp(-e)) < 2.0 / U32
    # smaller Gamma => stronger time coupling => fewer accepted breaks
    assert np.all(thr[0, :, 0] <= thr[-1, :, 0])


def test_swap_tables_closed_form_edges():
    beta, L_tau = 16.0, 256
    lad = np.array([2.0, 2.0, 2.5, 3.0])
    eq, ln, tabs = tables.swap_tables(beta, L_tau, lad)
    assert list(eq) == [1, 0, 0]
    assert ln[0] == 0
    for g in (1, 2):
        t = tabs[g].astype(np.int64)
        assert len(t) == ln[g] > 0
        assert np.all(np.diff(t) <= 0) and t[-1] > 0
        d = (-0.5 * math.log(math.tanh(beta * lad[g] / L_tau))
             + 0.5 * math.log(math.tanh(beta * lad[g + 1] / L_tau)))
        # the table ends where 2^32 e^{-4 m d} drops to at most 1
        m_end = len(t) + 1
        assert U32 * math.exp(-4 * m_end * d) <= 1.0 + 1e-6
        assert U32 * math.exp(-4 * (m_end - 1) * d) > 1.0 - 1e-6
    with pytest.raises(ValueError):
        tables.swap_tables(beta, L_tau, [3.0, 2.0])


# --------------------------------------------------------------------------
# Exact references cross-check each other
# --------------------------------------------------------------------------
def _lane0_couplings(L, seed):
    Jx, Jy = chain.couplings(L, [seed] * 64)
    jx = 1 - 2 * exact.bits_of_lane(Jx, 0)
    jy = 1 - 2 * exact.bits_of_lane(Jy, 0)
    return Jx, Jy, jx, jy


def test_enumeration_matches_transfer_matrix():
    _, _, jx, jy = _lane0_couplings(2, 5)
    k, kp = 0.25, 0.7
    e = exact.exact_moments(2, 4, jx, jy, k, kp)
    tm = exact.transfer_matrix_averages(jx, jy, 4, k, kp)
    assert abs(e["Bsp"] - tm["Bsp"]) < 1e-10
    assert abs(e["Bt"] - tm["Bt"]) < 1e-10


def test_classical_limit_of_enumeration():
    """Gamma -> 0: weights concentrate on tau-uniform configurations and
    <Bsp>/L_tau tends to the classical 2D +-J energy at beta."""
    _, _, jx, jy = _lane0_couplings(2, 9)
    beta, L_tau = 1.0, 4
    k = beta / L_tau
    kp = -0.5 * math.log(math.tanh(beta * 1e-6 / L_tau))
    e = exact.exact_moments(2, L_tau, jx, jy, k, kp)
    s = exact.spins_from_index(np.arange(16), 4)
    b, _ = exact.bond_sums(s, 2, 1, jx, jy)
    w = np.exp(beta * b - (beta * b).max())
    cl = float((w * b).sum() / w.sum())
    assert abs(e["Bsp"] / L_tau - cl) < 1e-6
    assert abs(e["Bt"] - 16) < 1e-6


# --------------------------------------------------------------------------
# Exact stationarity of the oracle's colour passes
# --------------------------------------------------------------------------
@pytest.mark.parametrize("beta,G", [(1.0, 1.0), (2.0, 3.0), (1.0, 0.4)])
def test_colour_pass_keeps_boltzmann_stationary(beta, G):
    """On L=2, L_tau=4 (2^16 states), build each colour pass's exact Markov
    operator from the oracle's own local classes and its table (acceptance
    (thr+1)/2^32); the Boltzmann distribution must be stationary up to the
    table quantisation (< 2^-32 per flip)."""
    L, L_tau = 2, 4
    Jx, Jy, jx, jy = _lane0_couplings(L, 3)
    k = beta / L_tau
    kp = -0.5 * math.log(math.tanh(beta * G / L_tau))
    idx, Bsp, Bt = exact.enumerate_states(L, L_tau, jx, jy)
    pi = exact.boltzmann(Bsp, Bt, k, kp)
    V = L * L * L_tau
    cfg = ((idx[:, None] >> np.arange(V)[None, :]) & 1).astype(np.uint64)
    ns, nt = chain.site_classes(L, L_tau, Jx, Jy, cfg.reshape(-1))
    thr = tables.metropolis_thresholds(beta, L_tau, [G])[0].astype(np.float64)
    p = (thr[ns, nt] + 1.0) / U32
    worst = 0.0
    for colour in (0, 1):
        out = exact.half_sweep_apply(pi, p, exact.colour_sites(L, L_tau, colour))
        worst = max(worst, float(np.max(np.abs(out - pi))))
    assert worst < 1e-8
    # the check has teeth: counting satisfied instead of unsatisfied time
    # bonds (a plausible index slip) breaks stationarity by far more
    bad = thr[:, ::-1].copy()
    pb = (bad[ns, nt] + 1.0) / U32
    dev = np.max(np.abs(exact.half_sweep_apply(pi, pb, exact.colour_sites(L, L_tau, 0)) - pi))
    assert dev > 1e-4


# --------------------------------------------------------------------------
# The chain itself: statistics against exact averages
# --------------------------------------------------------------------------
def _lane_means(og, n_sweeps, burn=200):
    og.run(burn, 0)
    acc_sp = np.zeros((og.N, 64))
    acc_t = np.zeros((og.N, 64))
    for _ in range(n_sweeps):
        og.run(1, 0)
        acc_sp += og.Bsp.reshape(og.N, 64)
        acc_t += og.Bt.reshape(og.N, 64)
    return acc_sp / n_sweeps, acc_t / n_sweeps


def _check_mean(lane_means, exact_value, nsig=5.0):
    m = lane_means.mean()
    se = lane_means.std(ddof=1) / math.sqrt(lane_means.size)
    assert abs(m - exact_value) < nsig * se + 1e-9, (m, exact_value, se)


@pytest.mark.parametrize("G", [0.6, 1.0])
def test_chain_trajectory_matches_exact_evolution_L2(G):
    """L=2, L_tau=4: for every lane, the expected time average of Bsp and Bt
    over the first T sweeps from that lane's initial state is computed
    exactly by evolving the observables with the exact sweep operator
    (2^16 states).  The chain's lane averages must agree within their
    spread.  No ergodicity is assumed (Metropolis accepts dE <= 0 with
    probability 1, and on this tiny lattice that leaves several closed
    classes, so long-run averages depend on the start)."""
    L, L_tau, beta, T = 2, 4, 1.0, 300
    Jx, Jy, jx, jy = _lane0_couplings(L, 3)
    idx, Bsp, Bt = exact.enumerate_states(L, L_tau, jx, jy)
    V = L * L * L_tau
    cfg = ((idx[:, None] >> np.arange(V)[None, :]) & 1).astype(np.uint64)
    ns, nt = chain.site_classes(L, L_tau, Jx, Jy, cfg.reshape(-1))
    thr = tables.metropolis_thresholds(beta, L_tau, [G])[0].astype(np.float64)
    p = (thr[ns, nt] + 1.0) / U32
    want_sp = exact.expected_time_average(Bsp, p, L, L_tau, T)
    want_t = exact.expected_time_average(Bt, p, L, L_tau, T)
    diffs_sp, diffs_t = [], []
    for rep in range(4):
        og = chain.OracleGroup(L, L_tau, beta, [G], rep, 42, [3] * 64)
        words = og.spins.copy()
        start = np.array([sum(int((int(words[s]) >> j) & 1) << s for s in range(V))
                          for j in range(64)])
        got_sp = np.zeros(64)
        got_t = np.zeros(64)
        for _ in range(T):
            og.run(1, 0)
            got_sp += og.Bsp
            got_t += og.Bt
        diffs_sp.append(got_sp / T - want_sp[start])
        diffs_t.append(got_t / T - want_t[start])
    for d in (np.concatenate(diffs_sp), np.concatenate(diffs_t)):
        se = d.std(ddof=1) / math.sqrt(d.size)
        assert abs(d.mean()) < 5 * se + 1e-9, (d.mean(), se)


def test_chain_matches_transfer_matrix_Ltau32():
    L, L_tau, beta, G = 2, 32, 4.0, 2.0
    _, _, jx, jy = _lane0_couplings(L, 11)
    og = chain.OracleGroup(L, L_tau, beta, [G], 0, 42, [11] * 64)
    msp, mt = _lane_means(og, 2000)
    k = beta / L_tau
    kp = -0.5 * math.log(math.tanh(beta * G / L_tau))
    tm = exact.transfer_matrix_averages(jx, jy, L_tau, k, kp)
    _check_mean(msp[0], tm["Bsp"])
    _check_mean(mt[0], tm["Bt"])


def test_decoupled_slices_are_classical_2d_metropolis():
    """kp -> 0 (large Gamma, every n_t class shares one threshold): the
    slices decouple into independent classical 2D +-J chains at coupling
    k.  On L=4 (2^16 states per slice) compare with exact enumeration."""
    L, L_tau, beta, G = 4, 2, 0.8, 60.0
    thr = tables.metropolis_thresholds(beta, L_tau, [G])[0]
    assert np.all(thr[:, 0] == thr[:, 1]) and np.all(thr[:, 1] == thr[:, 2])
    Jx, Jy, jx, jy = _lane0_couplings(L, 21)
    og = chain.OracleGroup(L, L_tau, beta, [G], 0, 42, [21] * 64)
    msp, _ = _lane_means(og, 3000)
    k = beta / L_tau
    s = exact.spins_from_index(np.arange(1 << 16), 16)
    b, _ = exact.bond_sums(s, L, 1, jx, jy)
    w = np.exp(k * b - (k * b).max())
    per_slice = float((w * b).sum() / w.sum())
    _check_mean(msp[0], L_tau * per_slice)


def test_tau_uniform_state_freezes_as_gamma_goes_to_zero():
    L, L_tau, beta, G = 4, 4, 1.0, 1e-6
    thr = tables.metropolis_thresholds(beta, L_tau, [G])[0]
    assert np.all(thr[:, 0] == 0)  # every break of two time bonds: r == 0 only
    V = L * L * L_tau
    rng = np.random.Generator(np.random.PCG64(0))
    plane = rng.integers(0, 2 ** 63, size=L * L, dtype=np.uint64)
    spins = np.tile(plane, L_tau)
    og = chain.OracleGroup(L, L_tau, beta, [G], 0, 42, [5] * 64, spins=spins)
    og.run(50, 0)
    assert np.array_equal(og.spins, spins)
    assert V == spins.size


def test_invariants_under_pt():
    for L, L_tau, ng, per_lane in ((4, 8, 3, False), (6, 4, 4, True), (2, 2, 2, False)):
        grp = W.tiny_group(L, L_tau, 1.5, ng, 0.5, 2.5, per_lane=per_lane)
        og = chain.OracleGroup.from_workload_group(grp)
        og.run(60, 5)  # raises if tracked and recomputed sums ever differ
        V = L * L * L_tau
        assert np.all((og.Bt - V) % 4 == 0)
        assert np.all(np.abs(og.Bsp) <= 2 * V)
        Bsp, Bt, _ = og.recompute()
        assert np.array_equal(Bsp.reshape(-1), og.Bsp)
        assert np.array_equal(Bt.reshape(-1), og.Bt)
        # one histogram entry per slot, lane and PT step; with L_tau slices
        # the unsatisfied time bonds of a lane are even, so only even u occur
        h = og.hist.reshape(ng, 1024)
        assert np.all(h.sum(axis=1) == og.p * 64)
        # walker labels stay a permutation of the slots in every lane
        wk = og.walker.reshape(ng, 64)
        assert np.all(np.sort(wk, axis=0) == np.arange(ng)[:, None])


def test_equal_gammas_rotate_walkers():
    """All Gammas equal: every exchange is accepted, so a sequential PT step
    carries the walker of slot 0 to slot N-1 and moves every other walker
    down one slot; a round trip then takes exactly N PT steps."""
    N = 5
    og = chain.OracleGroup(4, 4, 1.0, [1.3] * N, 0, 42, [1] * 64)
    steps = 40
    for p in range(steps):
        before = og.walker.reshape(N, 64).copy()
        og.pt_step()
        after = og.walker.reshape(N, 64)
        assert np.array_equal(after[N - 1], before[0])
        assert np.array_equal(after[:N - 1], before[1:])
    rows = og.swaplog_rows()
    assert np.all(rows == np.uint64(0xFFFFFFFFFFFFFFFF))
    cnt = og.rt_count.reshape(N, 64)
    tot = og.rt_sum.reshape(N, 64)
    assert cnt.sum() > 0
    assert np.all(tot[cnt > 0] == N * cnt[cnt > 0])


def test_swap_acceptance_frequency_matches_exchange_probability():
    """Start two slots with known Bt and measure how often the first PT
    step accepts: e^{(kp_0-kp_1) D} within binomial error."""
    L, L_tau, beta = 4, 8, 2.0
    lad = [1.0, 1.25]
    V = L * L * L_tau
    k_p = [-0.5 * math.log(math.tanh(beta * G / L_tau)) for G in lad]
    d = k_p[0] - k_p[1]
    # slot 0: all spins aligned (Bt = V); slot 1: site 0 alternates along
    # tau in every lane (Bt = V - 2 L_tau), so D = Bt1 - Bt0 = -2 L_tau
    s0 = np.zeros(V, dtype=np.uint64)
    s1 = np.zeros((L_tau, L * L), dtype=np.uint64)
    s1[1::2, 0] = np.uint64(0xFFFFFFFFFFFFFFFF)
    spins = np.concatenate([s0, s1.reshape(-1)])
    D = -2 * L_tau
    m = -D // 4
    p_exact = math.exp(-4 * m * d)
    accepted = 0
    trials = 0
    for rep in range(60):
        og = chain.OracleGroup(L, L_tau, beta, lad, rep, 42, [1] * 64, spins=spins)
        assert np.all(og.Bt.reshape(2, 64)[1] - og.Bt.reshape(2, 64)[0] == D)
        og.pt_step()
        mask = int(og.swaplog_rows()[0][0])
        accepted += bin(mask).count("1")
        trials += 64
    f = accepted / trials
    assert abs(f - p_exact) < 5 * math.sqrt(p_exact * (1 - p_exact) / trials)


@pytest.mark.slow
def test_pt_marginals_match_transfer_matrix():
    """Three slots on L=2, L_tau=32: with exchanges the chain still samples
    each slot's own Boltzmann distribution (exact per-slot averages from the
    transfer matrix)."""
    L, L_tau, beta = 2, 32, 4.0
    lad = [1.2, 2.0, 3.2]
    _, _, jx, jy = _lane0_couplings(L, 11)
    og = chain.OracleGroup(L, L_tau, beta, lad, 0, 42, [11] * 64)
    og.run(200, 2)
    n = 1500
    acc_t = np.zeros((3, 64))
    acc_sp = np.zeros((3, 64))
    for _ in range(n):
        og.run(2, 2)
        acc_t += og.Bt.reshape(3, 64)
        acc_sp += og.Bsp.reshape(3, 64)
    acc_t /= n
    acc_sp /= n
    k = beta / L_tau
    for g, G in enumerate(lad):
        kp = -0.5 * math.log(math.tanh(beta * G / L_tau))
        tm = exact.transfer_matrix_averages(jx, jy, L_tau, k, kp)
        _check_mean(acc_t[g], tm["Bt"])
        _check_mean(acc_sp[g], tm["Bsp"])
    assert og.acc.sum() > 0


# ------------------------------------------------------------------------
# Coupling ladder (one k on every bond, PT over k: the paper's Sec. 1
# parametrisation and Sec. 2.1 exchange with the full energy).

def test_k_ladder_thresholds_are_the_two_coupling_form_at_the_dual_field():
    """With beta/L_tau = k, the paper's relation Gamma = -ln tanh(k)/(2k)
    (Sec. 1) makes the time coupling -1/2 ln tanh(beta Gamma/L_tau) equal to
    k (the duality tanh(a) = e^{-2b} <=> tanh(b) = e^{-2a}), so each slot of
    a k ladder must have exactly the transverse-field table of that point;
    only three energy levels 4k, 8k, 12k occur (App. B's daemon levels)."""
    ks = W.linear_k_ladder(0.45, 0.2, 6)
    L_tau = 64
    thr_k = tables.metropolis_thresholds_k(ks)
    for g, k in enumerate(ks):
        gam = tables.gamma_of_equal_coupling(float(k))
        thr_g = tables.metropolis_thresholds(float(k) * L_tau, L_tau, [gam])[0]
        assert np.array_equal(thr_k[g], thr_g), g
        levels = sorted(set(int(x) for x in thr_k[g].reshape(-1)) - {2 ** 32 - 1})
        assert len(levels) == 3


def test_k_ladder_swap_frequency_uses_the_whole_energy():
    """Two k slots started with known Bsp and Bt: the first PT step accepts
    with frequency e^{(k_0-k_1) D}, D the change of Bsp + Bt (an exchange
    on Bt alone would give a visibly different rate)."""
    L, L_tau = 4, 8
    ks = [0.40, 0.34]
    V = L * L * L_tau
    s0 = np.zeros(V, dtype=np.uint64)
    s1 = np.zeros((L_tau, L * L), dtype=np.uint64)
    s1[1::2, 0] = np.uint64(0xFFFFFFFFFFFFFFFF)
    spins = np.concatenate([s0, s1.reshape(-1)])
    accepted = trials = 0
    D_all = D_t = None
    for rep in range(60):
        og = chain.OracleGroup(L, L_tau, 1.0, ks, rep, 42, [3] * 64, spins=spins, ladder="k")
        bsp = og.Bsp.reshape(2, 64)
        bt = og.Bt.reshape(2, 64)
        D = (bsp[1] + bt[1]) - (bsp[0] + bt[0])
        assert np.all(D == D[0])
        D_all, D_t = int(D[0]), int(bt[1][0] - bt[0][0])
        og.pt_step()
        accepted += bin(int(og.swaplog_rows()[0][0])).count("1")
        trials += 64
    assert D_all < 0 and D_all != D_t
    p_all = math.exp((ks[0] - ks[1]) * D_all)
    p_t = math.exp((ks[0] - ks[1]) * D_t)
    f = accepted / trials
    err = math.sqrt(p_all * (1 - p_all) / trials)
    assert abs(f - p_all) < 5 * err
    assert abs(f - p_t) > 5 * err


@pytest.mark.slow
def test_k_ladder_pt_marginals_match_transfer_matrix():
    """Three k slots on L=2, L_tau=32: with exchanges on the full energy each
    slot still samples its own Boltzmann weight e^{k_g (Bsp + Bt)} (exact
    per-slot averages from the transfer matrix at k = kp = k_g)."""
    L, L_tau = 2, 32
    ks = [0.55, 0.42, 0.30]
    _, _, jx, jy = _lane0_couplings(L, 11)
    og = chain.OracleGroup(L, L_tau, 1.0, ks, 0, 42, [11] * 64, ladder="k")
    og.run(200, 2)
    n = 1500
    acc_t = np.zeros((3, 64))
    acc_sp = np.zeros((3, 64))
    for _ in range(n):
        og.run(2, 2)
        acc_t += og.Bt.reshape(3, 64)
        acc_sp += og.Bsp.reshape(3, 64)
    acc_t /= n
    acc_sp /= n
    for g, k in enumerate(ks):
        tm = exact.transfer_matrix_averages(jx, jy, L_tau, k, k)
        _check_mean(acc_t[g], tm["Bt"])
        _check_mean(acc_sp[g], tm["Bsp"])
    assert og.acc.sum() > 0


def test_equal_k_rotate_walkers():
    """Equal couplings: every exchange is accepted whatever the energies."""
    N = 4
    og = chain.OracleGroup(4, 4, 1.0, [0.3] * N, 0, 42, [1] * 64, ladder="k")
    for _ in range(12):
        before = og.walker.reshape(N, 64).copy()
        og.pt_step()
        after = og.walker.reshape(N, 64)
        assert np.array_equal(after[N - 1], before[0])
        assert np.array_equal(after[:N - 1], before[1:])


# ------------------------------------------------------------------------
# Antiperiodic boundary along tau (Sec. 1: S(tau + L_tau) = -S(tau)).

def test_antiperiodic_enumeration_matches_transfer_matrix():
    _, _, jx, jy = _lane0_couplings(2, 5)
    for L_tau in (2, 4):
        e = exact.exact_moments(2, L_tau, jx, jy, 0.25, 0.7, antiperiodic=True)
        tm = exact.transfer_matrix_averages(jx, jy, L_tau, 0.25, 0.7, antiperiodic=True)
        assert abs(e["Bsp"] - tm["Bsp"]) < 1e-10
        assert abs(e["Bt"] - tm["Bt"]) < 1e-10
    # the twist matters: the periodic averages differ
    per = exact.exact_moments(2, 4, jx, jy, 0.25, 0.7)
    assert abs(per["Bt"] - e["Bt"]) > 1e-3


@pytest.mark.parametrize("beta,G", [(1.0, 1.0), (2.0, 3.0)])
def test_antiperiodic_colour_pass_keeps_boltzmann_stationary(beta, G):
    """As for the periodic prism: the exact colour-pass operators built from
    the oracle's own antiperiodic classes keep the antiperiodic Boltzmann
    weight stationary; the periodic classes do not."""
    L, L_tau = 2, 4
    Jx, Jy, jx, jy = _lane0_couplings(L, 3)
    k = beta / L_tau
    kp = -0.5 * math.log(math.tanh(beta * G / L_tau))
    idx, Bsp, Bt = exact.enumerate_states(L, L_tau, jx, jy, antiperiodic=True)
    pi = exact.boltzmann(Bsp, Bt, k, kp)
    V = L * L * L_tau
    cfg = ((idx[:, None] >> np.arange(V)[None, :]) & 1).astype(np.uint64)
    thr = tables.metropolis_thresholds(beta, L_tau, [G])[0].astype(np.float64)
    ns, nt = chain.site_classes(L, L_tau, Jx, Jy, cfg.reshape(-1), antiperiodic=True)
    p = (thr[ns, nt] + 1.0) / U32
    for colour in (0, 1):
        out = exact.half_sweep_apply(pi, p, exact.colour_sites(L, L_tau, colour))
        assert float(np.max(np.abs(out - pi))) < 1e-8
    ns0, nt0 = chain.site_classes(L, L_tau, Jx, Jy, cfg.reshape(-1))
    p0 = (thr[ns0, nt0] + 1.0) / U32
    dev = np.max(np.abs(exact.half_sweep_apply(pi, p0, exact.colour_sites(L, L_tau, 0)) - pi))
    assert dev > 1e-6  # far above the 1e-8 stationarity tolerance (weak kp at G = 3)


def test_antiperiodic_chain_matches_transfer_matrix_Ltau32():
    L, L_tau, beta, G = 2, 32, 4.0, 2.0
    _, _, jx, jy = _lane0_couplings(L, 11)
    og = chain.OracleGroup(L, L_tau, beta, [G], 0, 42, [11] * 64, antiperiodic=True)
    msp, mt = _lane_means(og, 2000)
    k = beta / L_tau
    kp = -0.5 * math.log(math.tanh(beta * G / L_tau))
    tm = exact.transfer_matrix_averages(jx, jy, L_tau, k, kp, antiperiodic=True)
    _check_mean(msp[0], tm["Bsp"])
    _check_mean(mt[0], tm["Bt"])
    # an odd number of unsatisfied time bonds in every tau column
    V = L * L * L_tau
    assert np.all(((V - og.Bt) // 2) % 2 == (L * L) % 2)


# ------------------------------------------------------------------------
# Euclidean-time overlaps (App. E): the oracle against definitions written
# out site by site, closed forms and symmetries.

def _random_words(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, 2 ** 63, size=n, dtype=np.int64).astype(np.uint64) * np.uint64(2) + \
        rng.integers(0, 2, size=n, dtype=np.int64).astype(np.uint64)


def test_tau_overlaps_match_site_by_site_definition():
    from oracle import overlaps
    L, L_tau = 3, 4
    words = _random_words(L * L * L_tau, 71)
    taus = [0, 1, 3]
    got = overlaps.contributions(words, L, L_tau, taus)
    for a in (0, 5, 63):
        spin = lambda x, y, t: -1 if (int(words[(t % L_tau) * L * L + y * L + x]) >> a) & 1 else 1
        for i, tau in enumerate(taus):
            q2 = q4 = 0
            for t1 in range(L_tau):
                Qt = sum(spin(x, y, t1) * spin(x, y, t1 + tau) for x in range(L) for y in range(L))
                q2 += Qt ** 2
                q4 += Qt ** 4
            assert got["q2"][a, i] == q2 and got["q4"][a, i] == q4
    # F through the integer correlations equals the complex sums
    i, tau = 1, 1
    direct = 0.0
    for a in range(64):
        for t1 in range(L_tau):
            for axis in (0, 1):
                z = 0j
                for x in range(L):
                    for y in range(L):
                        b1 = (int(words[t1 * L * L + y * L + x]) >> a) & 1
                        b2 = (int(words[((t1 + tau) % L_tau) * L * L + y * L + x]) >> a) & 1
                        q = 1 - 2 * (b1 ^ b2)
                        z += q * complex(math.cos(2 * math.pi * (x if axis == 0 else y) / L),
                                         math.sin(2 * math.pi * (x if axis == 0 else y) / L))
                direct += abs(z) ** 2
    w = np.array([math.cos(2 * math.pi * d / L) for d in range(L)])
    assert abs(float((got["A"][i] + got["B"][i]) @ w) - direct) < 1e-6 * direct


def test_tau_overlaps_closed_forms_and_symmetry():
    from oracle import overlaps
    L, L_tau = 4, 8
    words = _random_words(L * L * L_tau, 5)
    taus = list(range(L_tau))
    c = overlaps.contributions(words, L, L_tau, taus)
    # tau = 0: every q is 1
    assert np.all(c["q2"][:, 0] == L_tau * L ** 4)
    assert np.all(c["q4"][:, 0] == L_tau * L ** 8)
    assert np.all(c["A"][0] == 64 * L_tau * L ** 3) and np.all(c["B"][0] == 64 * L_tau * L ** 3)
    obs = overlaps.observables(c, L, L_tau, 1)
    assert abs(obs["F"][0]) < 1e-9 and abs(obs["Q2"][0] - L ** 4) < 1e-9
    # Qt(tau1, tau) = Qt(tau1 + tau, L_tau - tau): sums over tau1 agree
    for tau in range(1, L_tau):
        assert np.array_equal(c["q2"][:, tau], c["q2"][:, L_tau - tau])
        assert np.array_equal(c["q4"][:, tau], c["q4"][:, L_tau - tau])
        assert np.array_equal(c["A"][tau], c["A"][L_tau - tau])
    # independent random spins: <Qt^2> = L^2 away from tau = 0
    m = c["q2"][:, 1:].mean() / L_tau
    assert abs(m - L * L) < 0.1 * L * L


# ------------------------------------------------------------------------
# Measurements of App. A / App. E taken at every PT step: the same-time,
# same-tau replica overlap q of lane pairs (2p, 2p+1) and the histogram of
# unsatisfied time bonds.  Each expected value is built by hand from a
# configuration whose answer is known, not by re-running the oracle's sums.

def _pair_spins(V, even_words, relation):
    """Words whose odd lanes are built from the even lanes: relation[p] is
    'same' (lane 2p+1 = lane 2p) or 'flip' (lane 2p+1 = -lane 2p) for the
    32 pairs."""
    out = np.zeros(V, dtype=np.uint64)
    for s in range(V):
        w = int(even_words[s])
        word = 0
        for p in range(32):
            b = (w >> (2 * p)) & 1
            ob = b if relation[p] == "same" else 1 - b
            word |= (b << (2 * p)) | (ob << (2 * p + 1))
        out[s] = word
    return out


def test_overlap_of_identical_and_complementary_pairs():
    """q_p = sum over sites of S^{2p} S^{2p+1} (App. E, tau1 = tau2, t1 = t2):
    +V for identical lanes and -V for complementary ones, whatever the
    configuration; pairing any other two lanes (say p and p+32) would give
    values near 0 for these random words."""
    L, L_tau = 4, 6
    V = L * L * L_tau
    rel = ["same" if p % 3 else "flip" for p in range(32)]
    spins = _pair_spins(V, _random_words(V, 11), rel)
    og = chain.OracleGroup(L, L_tau, 1.0, [1.0], 0, 42, [1] * 64, spins=spins)
    _, _, q = og.recompute()
    want = np.array([V if r == "same" else -V for r in rel])
    assert np.array_equal(q[0], want)


def test_overlap_counts_differing_sites():
    """Pair p differs on exactly d_p chosen sites: q_p = V - 2 d_p."""
    L, L_tau = 4, 4
    V = L * L * L_tau
    rng = np.random.Generator(np.random.PCG64(12))
    base = _pair_spins(V, _random_words(V, 13), ["same"] * 32)
    d = rng.integers(0, V + 1, size=32)
    spins = base.copy()
    for p in range(32):
        for s in rng.choice(V, size=int(d[p]), replace=False):
            spins[s] ^= np.uint64(1 << (2 * p + 1))
    og = chain.OracleGroup(L, L_tau, 1.0, [1.0, 1.5], 0, 42, [1] * 64,
                           spins=np.concatenate([spins, base]))
    _, _, q = og.recompute()
    assert np.array_equal(q[0], V - 2 * d)
    assert np.all(q[1] == V)
    # the PT step adds q and q^2 of the configuration before any exchange
    og.pt_step()
    assert np.array_equal(og.sum_q.reshape(2, 32)[0], V - 2 * d)
    assert np.array_equal(og.sum_q2.reshape(2, 32)[0], (V - 2 * d) ** 2)


def test_overlap_of_independent_lanes_has_variance_V():
    """Independent uniform spins: q_p is a sum of V independent +-1, so
    <q> = 0 and <q^2> = V."""
    L, L_tau = 4, 8
    V = L * L * L_tau
    qs = []
    for seed in range(40):
        og = chain.OracleGroup(L, L_tau, 1.0, [1.0], 0, 42, [1] * 64,
                               spins=_random_words(V, 100 + seed))
        qs.append(og.recompute()[2][0])
    q = np.concatenate(qs).astype(np.float64)
    n = q.size
    assert abs(q.mean()) < 5 * math.sqrt(V / n)
    # var(q^2) = 3V^2 - 2V for sums of independent +-1
    assert abs((q * q).mean() - V) < 5 * math.sqrt((2 * V * V - 2 * V) / n)


def _columns_with_breaks(L, L_tau, breaks_per_lane):
    """Configuration (one slot) in which lane j has exactly
    breaks_per_lane[j] unsatisfied time bonds: column c of the plane flips
    sign after slice 0 and back after slice b_c (two breaks per flipped
    column; the count of a periodic ring is even)."""
    P = L * L
    words = np.zeros((L_tau, P), dtype=np.uint64)
    for j, u in enumerate(breaks_per_lane):
        assert u % 2 == 0 and u // 2 <= P
        for c in range(u // 2):
            b = 1 + (c % (L_tau - 1))
            for t in range(1, b + 1):
                words[t, c] |= np.uint64(1 << j)
    return words.reshape(-1)


def test_unsatisfied_time_bond_histogram_bins():
    """Lane j with u_j unsatisfied time bonds is counted in bin
    u_j * 1024 // (V + 1) of its slot at a PT step; u is counted here
    directly from the words, bond by bond."""
    for L, L_tau in ((2, 4), (4, 8)):
        V = L * L * L_tau
        rng = np.random.Generator(np.random.PCG64(V))
        u = 2 * rng.integers(0, L * L + 1, size=64)
        u[0], u[1] = 0, 2 * L * L  # both ends of the range
        cfg = _columns_with_breaks(L, L_tau, u)
        cfg2 = _random_words(V, 21)
        og = chain.OracleGroup(L, L_tau, 1.0, [1.0, 2.0], 0, 42, [1] * 64,
                               spins=np.concatenate([cfg, cfg2]))
        og.pt_step()
        h = og.hist.reshape(2, 1024)
        for slot, words in ((0, cfg), (1, cfg2)):
            w = words.reshape(L_tau, L * L)
            direct = np.zeros(64, dtype=np.int64)
            for t in range(L_tau):
                diff = w[t] ^ w[(t + 1) % L_tau]
                for j in range(64):
                    direct[j] += int(sum((int(x) >> j) & 1 for x in diff))
            if slot == 0:
                assert np.array_equal(direct, u)
            want = np.zeros(1024, dtype=np.int64)
            for j in range(64):
                want[direct[j] * 1024 // (V + 1)] += 1
            assert np.array_equal(h[slot], want), (L, L_tau, slot)


def test_one_slot_group_is_measured_without_exchanges():
    """A one-slot group has no exchange partner: a PT step exchanges nothing
    and counts no round trip, but its energies, overlaps and histogram are
    measured like any other slot's (App. A)."""
    og = chain.OracleGroup(4, 4, 1.0, [1.0], 0, 42, [1] * 64)
    og.run(30, 10)
    assert og.p == 3
    assert np.all(og.hist.sum() == 3 * 64)
    assert np.all(og.rt_count == 0)
    assert np.all(og.walker == 0)
    Bsp, Bt, q = og.recompute()
    assert np.any(og.sum_Bt != 0) and np.any(og.sum_q2 != 0)


# ------------------------------------------------------------------------
# Lane numbers of the Metropolis test: bit (31 - b) of lane j's r is bit j
# of level b, level 2q = o0 | o1 << 32 and level 2q+1 = o2 | o3 << 32 of
# the Philox block with counter (s, t, (g << 4) | q, group_id).  The three
# published known-answer vectors fix two levels each without running any
# generator code.

def _levels_from_kat(o):
    return (int(o[0]) | int(o[1]) << 32, int(o[2]) | int(o[3]) << 32)


@pytest.mark.parametrize("row", range(3))
def test_metropolis_levels_from_published_philox_outputs(philox_kat, row):
    ctr, key, out = philox_kat[row]
    s, t, c2, gid = ctr
    seed = key[0] | key[1] << 32
    g, q = c2 >> 4, c2 & 15  # counter word 2 = (g << 4) | q in domain 0
    lv = _levels_from_kat(out)
    r = chain.metropolis_r(seed, gid, s, t, g)
    for j in range(64):
        for h in (0, 1):
            b = 2 * q + h
            assert (int(r[j]) >> (31 - b)) & 1 == (lv[h] >> j) & 1, (row, j, b)


def test_pt_number_from_published_philox_output(philox_kat):
    """PT numbers: word j & 3 of the block with counter (j >> 2, p,
    (1 << 24) | g, group_id); the third known-answer vector has a counter
    word 2 whose bit 24 is set, so it is the block of pair g = that word."""
    ctr, key, out = philox_kat[2]
    assert (ctr[2] >> 24) & 1
    seed = key[0] | key[1] << 32
    for w in range(4):
        j = (ctr[0] << 2) | w
        assert chain.pt_r(seed, ctr[3], ctr[1], ctr[2], j) == out[w]


def test_lane_numbers_are_independent_across_lanes():
    """Different lanes draw different numbers: over many (s, t, g) no two
    lanes of a word share r, and every pair of lanes agrees on the top bit
    half of the time (a level assembled from one output word twice, or a
    lane read twice, makes two lanes equal)."""
    rs = np.stack([chain.metropolis_r(7, 3, s, t, g)
                   for s in range(60) for t in range(4) for g in range(2)])
    n = rs.shape[0]
    for row in rs:
        assert len(set(int(x) for x in row)) == 64
    top = (rs >> np.uint32(31)).astype(np.int64)
    agree = (top[:, :, None] == top[:, None, :]).mean(axis=0)
    off = agree[~np.eye(64, dtype=bool)]
    assert np.all(np.abs(off - 0.5) < 6 * math.sqrt(0.25 / n))
    low = (rs & np.uint32(0xFF)).astype(np.int64)
    corr = np.corrcoef(low.T)[~np.eye(64, dtype=bool)]
    assert np.all(np.abs(corr) < 6 / math.sqrt(n))


# ------------------------------------------------------------------------
# Exact quantisation thr = ceil(2^32 p) - 1, i.e. thr < 2^32 p <= thr + 1
# (accept <=> r < 2^32 p for a uniform 32-bit r).  Checked in double where
# 2^32 p is not within 1e-3 of an integer, so that floor, round or an
# off-by-one each fail on a good share of the entries.

def _check_quantised(thr, x):
    frac = x - math.floor(x)
    if 1e-3 < frac < 1 - 1e-3:
        assert thr == math.ceil(x) - 1, (thr, x)
        return 1
    return 0


@pytest.mark.parametrize("beta,L_tau,lo,hi,n", [(8.0, 128, 2.0, 4.0, 32), (4.0, 32, 1.5, 4.5, 16),
                                               (128.0, 2048, 2.8, 3.6, 48), (1.0, 8, 0.2, 0.9, 6)])
def test_metropolis_thresholds_are_ceil_of_scaled_probability(beta, L_tau, lo, hi, n):
    lad = W.geometric_ladder(lo, hi, n)
    thr = tables.metropolis_thresholds(beta, L_tau, lad)
    k = beta / L_tau
    checked = 0
    for g, G in enumerate(lad):
        kp = -0.5 * math.log(math.tanh(beta * G / L_tau))
        for ns in range(5):
            for nt in range(3):
                dE = 4 * k * (2 - ns) + 4 * kp * (1 - nt)
                if dE <= 0:
                    assert int(thr[g, ns, nt]) == U32 - 1
                    continue
                checked += _check_quantised(int(thr[g, ns, nt]), U32 * math.exp(-dE))
    assert checked >= 4 * n


def test_exchange_thresholds_are_ceil_of_scaled_probability():
    beta, L_tau = 16.0, 256
    lad = W.geometric_ladder(2.0, 4.0, 12)
    eq, ln, tabs = tables.swap_tables(beta, L_tau, lad)
    checked = 0
    for g in range(len(lad) - 1):
        d = (-0.5 * math.log(math.tanh(beta * lad[g] / L_tau))
             + 0.5 * math.log(math.tanh(beta * lad[g + 1] / L_tau)))
        for m in range(1, int(ln[g]) + 1, 7):
            checked += _check_quantised(int(tabs[g][m - 1]), U32 * math.exp(-4 * m * d))
    assert checked > 100
