"""Euclidean-time overlaps of one slot's configuration (test oracle).

TEST INFRASTRUCTURE ONLY: used by the tests, never by the product.

Paper, App. E (the `overlap_tau` quantities): for replica a at Monte Carlo
time t, q_x(tau1, tau) = S_{x,tau1} S_{x,tau1+tau} (tau1 + tau taken modulo
L_tau: the quantities are even in q, so periodic and antiperiodic prisms
give the same values) and Qt(tau1, tau) = sum_x q_x.  From them

    Q2(tau) = < Qt^2 >,  Q4(tau) = < Qt^4 >,
    F(tau)  = < |sum_x e^{i 2 pi x1 / L} q_x|^2 + |sum_x e^{i 2 pi x2 / L} q_x|^2 > / 2,

averages over tau1, Monte Carlo time and replicas.  What one configuration
contributes, kept as integers so that sums are exact and independent of
order:

    q2[a][i] = sum_tau1 Qt^2,  q4[a][i] = sum_tau1 Qt^4       (tau = taus[i])
    A[i][d]  = sum_{a, tau1} sum_{x1} C_{x1} C_{x1+d},  C_{x1} = sum_{x2} q_{x1,x2}
    B[i][d]  = the same with R_{x2} = sum_{x1} q_{x1,x2}

and |sum_x e^{i 2 pi x1/L} q_x|^2 = sum_d A-term(d) cos(2 pi d / L).
x1 is the column (x) and x2 the row (y) coordinate of the plane.
"""
from __future__ import annotations

import math
from typing import Dict, Sequence

import numpy as np


def lane_spins(words: np.ndarray, L: int, L_tau: int) -> np.ndarray:
    """+-1 spins [64][L_tau][L (y)][L (x)] of a slot's words [L_tau][L][L]."""
    w = np.asarray(words, dtype=np.uint64).reshape(L_tau, L, L)
    bits = (w[None] >> np.arange(64, dtype=np.uint64)[:, None, None, None]) & np.uint64(1)
    return 1 - 2 * bits.astype(np.int64)


def contributions(words: np.ndarray, L: int, L_tau: int, taus: Sequence[int]) -> Dict[str, np.ndarray]:
    S = lane_spins(words, L, L_tau)                     # [a][tau][y][x]
    n = len(taus)
    q2 = np.zeros((64, n), dtype=np.int64)
    q4 = np.zeros((64, n), dtype=np.int64)
    A = np.zeros((n, L), dtype=np.int64)
    B = np.zeros((n, L), dtype=np.int64)
    for i, tau in enumerate(taus):
        q = S * np.roll(S, -int(tau), axis=1)           # q[a][tau1][y][x]
        Qt = q.sum(axis=(2, 3))                         # [a][tau1]
        q2[:, i] = (Qt ** 2).sum(axis=1)
        q4[:, i] = (Qt ** 4).sum(axis=1)
        C = q.sum(axis=2)                               # column sums over y: [a][tau1][x1]
        R = q.sum(axis=3)                               # row sums over x: [a][tau1][x2]
        for d in range(L):
            A[i, d] = int((C * np.roll(C, -d, axis=2)).sum())
            B[i, d] = int((R * np.roll(R, -d, axis=2)).sum())
    return {"q2": q2, "q4": q4, "A": A, "B": B}


def observables(acc: Dict[str, np.ndarray], L: int, L_tau: int, n_configs: int) -> Dict[str, np.ndarray]:
    """Q2(tau), Q4(tau), F(tau) per the paper's normalisation (averaged over
    tau1, configurations and the 64 replicas), from summed contributions."""
    norm = float(L_tau) * n_configs
    w = np.array([math.cos(2 * math.pi * d / L) for d in range(L)])
    Q2 = acc["q2"].astype(np.float64).mean(axis=0) / norm
    Q4 = acc["q4"].astype(np.float64).mean(axis=0) / norm
    F = ((acc["A"] + acc["B"]).astype(np.float64) @ w) / (2.0 * norm * 64)
    return {"Q2": Q2, "Q4": Q4, "F": F}
