"""Exact results that pin the oracle chain (test infrastructure).

Everything here is written from the definitions, independently of the C
chain:

* `enumerate_states`: every configuration of a tiny prism (2^(L^2 L_tau)
  states), its bond sums and Boltzmann weights exp(k Bsp + kp Bt) of the
  Trotter-Suzuki form (paper: Sec. 1, Eqs. (2)-(3), with separate space and
  time couplings).
* `transfer_matrix_averages`: the same averages for L = 2 and any L_tau from
  the slice transfer matrix T = e^{k b(S)/2} e^{kp S.S'} e^{k b(S')/2}
  (paper: Sec. 2.2, the symmetric transfer matrix, in its classical form).
* `half_sweep_apply` / `half_sweep_backward`: the exact Markov operator of
  one colour pass of the checkerboard Metropolis update (Sec. 2.1), with the
  quantised acceptance (thr+1)/2^32 of the integer test r <= thr, acting on
  distributions and on observables.
"""
from __future__ import annotations

from typing import Dict

import numpy as np


def bits_of_lane(words: np.ndarray, lane: int) -> np.ndarray:
    return ((np.asarray(words, dtype=np.uint64) >> np.uint64(lane)) & np.uint64(1)).astype(np.int64)


def spins_from_index(idx: np.ndarray, V: int) -> np.ndarray:
    """[n, V] array of +-1; bit s of the index set <=> S_s = -1."""
    b = (idx[:, None] >> np.arange(V)[None, :]) & 1
    return 1 - 2 * b


def bond_sums(S: np.ndarray, L: int, L_tau: int, jx: np.ndarray, jy: np.ndarray,
              antiperiodic: bool = False):
    """Bsp and Bt of configurations S [n, V] (site s = x + L(y + L tau)).

    jx, jy: +-1 couplings [L*L] of the +x and +y bonds of site (x,y).
    antiperiodic: S(tau + L_tau) = -S(tau), i.e. the bond from the last slice
    to the first counts with the opposite sign."""
    n = S.shape[0]
    S4 = S.reshape(n, L_tau, L, L)  # [n][tau][y][x]
    Jx = jx.reshape(L, L)[None, None]  # [y][x]
    Jy = jy.reshape(L, L)[None, None]
    Bsp = (Jx * S4 * np.roll(S4, -1, axis=3)).sum(axis=(1, 2, 3)) + \
          (Jy * S4 * np.roll(S4, -1, axis=2)).sum(axis=(1, 2, 3))
    up = np.roll(S4, -1, axis=1)
    if antiperiodic:
        up[:, L_tau - 1] *= -1
    Bt = (S4 * up).sum(axis=(1, 2, 3))
    return Bsp.astype(np.int64), Bt.astype(np.int64)


def enumerate_states(L: int, L_tau: int, jx, jy, antiperiodic: bool = False):
    V = L * L * L_tau
    assert V <= 20
    idx = np.arange(1 << V, dtype=np.int64)
    S = spins_from_index(idx, V)
    Bsp, Bt = bond_sums(S, L, L_tau, np.asarray(jx), np.asarray(jy), antiperiodic)
    return idx, Bsp, Bt


def boltzmann(Bsp, Bt, k: float, kp: float) -> np.ndarray:
    e = k * Bsp + kp * Bt
    w = np.exp(e - e.max())
    return w / w.sum()


def exact_moments(L, L_tau, jx, jy, k, kp, antiperiodic: bool = False) -> Dict[str, float]:
    _, Bsp, Bt = enumerate_states(L, L_tau, jx, jy, antiperiodic)
    w = boltzmann(Bsp, Bt, k, kp)
    return {
        "Bsp": float((w * Bsp).sum()),
        "Bt": float((w * Bt).sum()),
        "Bsp2": float((w * Bsp * Bsp).sum()),
        "Bt2": float((w * Bt * Bt).sum()),
    }


def transfer_matrix_averages(jx, jy, L_tau: int, k: float, kp: float,
                             L: int = 2, antiperiodic: bool = False) -> Dict[str, float]:
    """<Bsp>, <Bt> for an L x L lattice with L_tau slices, periodic in tau
    (or antiperiodic: the last transfer step carries e^{-kp S.S'}; moving the
    twist to another bond is a change of variables, so every slice and every
    time bond, counted with its sign, has the same average)."""
    n = L * L
    idx = np.arange(1 << n)
    s = spins_from_index(idx, n)  # slice states [2^n, n]
    b, _ = bond_sums(s, L, 1, np.asarray(jx), np.asarray(jy))
    # _ (the time sum of a one-slice prism) is not used
    ov = s @ s.T  # sum_x S_x S'_x
    half = np.exp(0.5 * k * b)
    T = half[:, None] * np.exp(kp * ov) * half[None, :]
    Tw = half[:, None] * np.exp(-kp * ov) * half[None, :] if antiperiodic else T
    Tn2 = np.linalg.matrix_power(T, L_tau - 2)
    Tn1 = Tn2 @ Tw  # every step but the first, the twisted one last
    Tn = T @ Tn1
    Z = np.trace(Tn)
    Bsp = L_tau * np.trace(np.diag(b.astype(float)) @ Tn) / Z
    Bt = L_tau * np.trace((T * ov) @ Tn1) / Z
    return {"Bsp": float(Bsp), "Bt": float(Bt), "Z": float(Z)}


def colour_sites(L: int, L_tau: int, colour: int):
    out = []
    for tau in range(L_tau):
        for y in range(L):
            for x in range(L):
                if (x + y + tau) % 2 == colour:
                    out.append(x + L * (y + L * tau))
    return out


def half_sweep_apply(pi: np.ndarray, flip_prob: np.ndarray, sites) -> np.ndarray:
    """Apply the colour-pass operator to a distribution over states.

    flip_prob[state, site] = acceptance probability of flipping that site in
    that state.  Sites of one colour do not interact, so the pass is the
    product of the single-site operators, applied one after the other."""
    out = pi.copy()
    idx = np.arange(pi.size)
    for s in sites:
        p = flip_prob[:, s]
        partner = idx ^ (1 << s)
        out = out * (1.0 - p) + out[partner] * p[partner]
    return out


def half_sweep_backward(f: np.ndarray, flip_prob: np.ndarray, sites) -> np.ndarray:
    """Apply a colour pass to an observable: (K f)(S) = E[f(S') | S].

    Used to get exact expectations along a trajectory from a given start
    without assuming the chain is irreducible (with acceptance 1 for
    dE <= 0, Metropolis on a tiny lattice can have several closed classes)."""
    out = f.copy()
    idx = np.arange(f.size)
    for s in reversed(list(sites)):
        p = flip_prob[:, s]
        out = (1.0 - p) * out + p * out[idx ^ (1 << s)]
    return out


def expected_time_average(f: np.ndarray, flip_prob: np.ndarray, L: int,
                          L_tau: int, n_sweeps: int) -> np.ndarray:
    """For every start state S0: (1/T) sum_{t=1..T} E[f(S_t) | S0], one sweep
    being the red pass followed by the blue pass."""
    red = colour_sites(L, L_tau, 0)
    blue = colour_sites(L, L_tau, 1)
    g = f.astype(np.float64)
    acc = np.zeros_like(g)
    for _ in range(n_sweeps):
        # E[f(S_t)|S0] = K_red K_blue applied t times; red acts first in time,
        # so on observables it is applied last
        g = half_sweep_backward(half_sweep_backward(g, flip_prob, blue), flip_prob, red)
        acc += g
    return acc / n_sweeps
