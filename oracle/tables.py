"""Metropolis and parallel-tempering thresholds, in mpmath (test oracle).

Paper: Sec. 2.1 precomputes the Metropolis factor e^{-k (E'-E)} for every
possible energy change; App. C builds its random-number tables in 128-bit
floating point.  Here the factors become uint32 thresholds, exact for the
comparison that the chain performs:

    accept  <=>  r < 2^32 * min(1, e^{-dE})  <=>  r <= ceil(2^32 min(1,e^{-dE})) - 1

for a uniform 32-bit integer r.  dE is computed from the exact values of the
double inputs beta, Gamma_g and the integer L_tau at 50 decimal digits.

Two-coupling Trotter-Suzuki form: k = beta/L_tau on space bonds,
kp_g = -1/2 ln tanh(beta Gamma_g / L_tau) on time bonds.  A spin with n_s
unsatisfied space bonds (of 4) and n_t unsatisfied time bonds (of 2) changes
the exponent of its weight by dE = 4k(2-n_s) + 4kp(1-n_t) when flipped.

Exchange of the configurations at slots g and g+1 (Sec. 2.1, the parallel
tempering exchange probability): with D = Bt[g+1]-Bt[g] (a multiple of 4),
P = min(1, e^{(kp_g - kp_{g+1}) D}).  For D = -4m the threshold is
ceil(2^32 e^{-4 m (kp_g-kp_{g+1})}) - 1; the table of pair g lists m = 1..len
while the threshold is positive, and is 0 beyond.

The coupling-ladder form (one k_g on every bond of slot g) is at the end.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import mpmath
import numpy as np

DPS = 50
TWO32 = 2 ** 32
U32MAX = TWO32 - 1


def _ctx():
    ctx = mpmath.mp.clone()
    ctx.dps = DPS
    return ctx


def couplings(beta: float, L_tau: int, gammas: Sequence[float]):
    """(k, [kp_g]) as mpmath numbers."""
    mp = _ctx()
    k = mp.mpf(float(beta)) / L_tau
    kps = [-mp.log(mp.tanh(mp.mpf(float(beta)) * mp.mpf(float(G)) / L_tau)) / 2
           for G in gammas]
    return mp, k, kps


def _thr_of_exponent(mp, x) -> int:
    """ceil(2^32 * min(1, e^{-x})) - 1 for an mpmath exponent x."""
    if x <= 0:
        return U32MAX
    v = int(mp.ceil(mp.ldexp(mp.exp(-x), 32))) - 1
    return max(0, min(U32MAX, v))


def metropolis_thresholds(beta: float, L_tau: int,
                          gammas: Sequence[float]) -> np.ndarray:
    """uint32 [N][5][3]: thr[g][n_s][n_t]."""
    mp, k, kps = couplings(beta, L_tau, gammas)
    out = np.zeros((len(gammas), 5, 3), dtype=np.uint32)
    for g, kp in enumerate(kps):
        for ns in range(5):
            for nt in range(3):
                dE = 4 * k * (2 - ns) + 4 * kp * (1 - nt)
                out[g, ns, nt] = _thr_of_exponent(mp, dE)
    return out


def swap_tables(beta: float, L_tau: int, gammas: Sequence[float],
                cap: int = 1 << 20) -> Tuple[np.ndarray, np.ndarray, List[np.ndarray]]:
    """Returns (equal[N-1] uint8, length[N-1] uint32, [entries per pair]).

    equal[g] = 1 when Gamma_g == Gamma_{g+1} (then kp_g == kp_{g+1} exactly
    and every exchange is accepted).  The ladder must be non-decreasing.
    """
    n = len(gammas)
    for g in range(n - 1):
        if not float(gammas[g]) <= float(gammas[g + 1]):
            raise ValueError("ladder must be non-decreasing")
    mp, k, kps = couplings(beta, L_tau, gammas)
    equal = np.zeros(n - 1, dtype=np.uint8)
    lens = np.zeros(n - 1, dtype=np.uint32)
    tabs: List[np.ndarray] = []
    for g in range(n - 1):
        if float(gammas[g]) == float(gammas[g + 1]):
            equal[g] = 1
            tabs.append(np.zeros(0, dtype=np.uint32))
            continue
        d = kps[g] - kps[g + 1]
        ent = []
        m = 1
        while True:
            v = _thr_of_exponent(mp, 4 * m * d)
            if v == 0:
                break
            ent.append(v)
            m += 1
            if m > cap:
                raise ValueError("swap table longer than cap")
        lens[g] = len(ent)
        tabs.append(np.array(ent, dtype=np.uint32))
    return equal, lens, tabs


def flat_swap_tables(beta, L_tau, gammas):
    equal, lens, tabs = swap_tables(beta, L_tau, gammas)
    offs = np.zeros(len(lens), dtype=np.uint64)
    acc = 0
    for g, t in enumerate(tabs):
        offs[g] = acc
        acc += len(t)
    flat = np.concatenate(tabs).astype(np.uint32) if acc else np.zeros(1, np.uint32)
    return equal, lens, offs, flat


# --------------------------------------------------------------------------
# Coupling ladder (the paper's own parametrisation, Sec. 1 Eqs. (2)-(3)): slot
# g has one coupling k_g on every bond, so dE = 4k_g(2-n_s) + 4k_g(1-n_t);
# the exchange (Sec. 2.1) uses the full energy, P = min(1, e^{(k_g-k_{g+1}) D})
# with D = B[g+1]-B[g], B = Bsp + Bt.  The k list is non-increasing (App. C
# lists it in decreasing order).

def metropolis_thresholds_k(ks: Sequence[float]) -> np.ndarray:
    """uint32 [N][5][3]: thr[g][n_s][n_t] for couplings k_g."""
    mp = _ctx()
    out = np.zeros((len(ks), 5, 3), dtype=np.uint32)
    for g, kf in enumerate(ks):
        k = mp.mpf(float(kf))
        for ns in range(5):
            for nt in range(3):
                out[g, ns, nt] = _thr_of_exponent(mp, 4 * k * (2 - ns) + 4 * k * (1 - nt))
    return out


def swap_tables_k(ks: Sequence[float], cap: int = 1 << 20):
    """(equal[N-1], length[N-1], [entries per pair]) for a coupling ladder."""
    n = len(ks)
    for g in range(n - 1):
        if not float(ks[g]) >= float(ks[g + 1]):
            raise ValueError("k ladder must be non-increasing")
    mp = _ctx()
    equal = np.zeros(max(n - 1, 0), dtype=np.uint8)
    lens = np.zeros(max(n - 1, 0), dtype=np.uint32)
    tabs: List[np.ndarray] = []
    for g in range(n - 1):
        if float(ks[g]) == float(ks[g + 1]):
            equal[g] = 1
            tabs.append(np.zeros(0, dtype=np.uint32))
            continue
        d = mp.mpf(float(ks[g])) - mp.mpf(float(ks[g + 1]))
        ent = []
        m = 1
        while True:
            v = _thr_of_exponent(mp, 4 * m * d)
            if v == 0:
                break
            ent.append(v)
            m += 1
            if m > cap:
                raise ValueError("swap table longer than cap")
        lens[g] = len(ent)
        tabs.append(np.array(ent, dtype=np.uint32))
    return equal, lens, tabs


def flat_swap_tables_k(ks):
    equal, lens, tabs = swap_tables_k(ks)
    offs = np.zeros(len(lens), dtype=np.uint64)
    acc = 0
    for g, t in enumerate(tabs):
        offs[g] = acc
        acc += len(t)
    flat = np.concatenate(tabs).astype(np.uint32) if acc else np.zeros(1, np.uint32)
    return equal, lens, offs, flat


def gamma_of_equal_coupling(k: float) -> float:
    """Gamma with kp == k: the paper's relation Gamma = -ln tanh(k) / (2k)
    (Sec. 1), evaluated for beta/L_tau = k."""
    mp = _ctx()
    kk = mp.mpf(k)
    return float(-mp.log(mp.tanh(kk)) / (2 * kk))
