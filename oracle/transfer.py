"""Transfer matrix of the Trotter-Suzuki form in its parity sectors (test oracle).

TEST INFRASTRUCTURE ONLY: used by the tests and the bench's CPU baseline,
never by the product.

Paper: Sec. 2.2 (the EDQSG code: the transfer matrix, the matrix-free
product in three phases, the XOR-stride rounds) and App. D (the
parity-aware basis).
For an L x L slice with couplings J and the two couplings of the Trotter
form (space k, time kp; the paper's equal-coupling form is kp = k):

    T = W B W,   W = diag exp(k Bsp(S) / 2),
    B = prod_sites (jp 1 + jm sigma^X_j),   jp = e^kp / (e^kp + e^-kp),
                                            jm = e^-kp / (e^kp + e^-kp),

i.e. T[S, S'] = e^{k Bsp(S)/2} prod_j (jp if S_j = S'_j else jm) e^{k Bsp(S')/2},
the classical slice transfer matrix divided by (2 cosh kp)^(L^2).  Bsp(S)
is the sum over the 2 L^2 bonds (site, +x) and (site, +y) of J S S'
(site j = x1 + L x2; bit j of a state index set means S_j = -1).

The parity P = prod_j sigma^X_j commutes with T.  With n an (L^2 - 1)-bit
index (the last site's spin fixed to +1), the sector bases are
|n>_e,o = (|n> +- |~n>) / sqrt(2), ~n the complement of all L^2 bits.  From
the matrix elements above, <m|B|n> = prod_{j < L^2-1} F[m_j][n_j] times jp
(the last site agrees) and <m|B|~n> = prod_{j < L^2-1} F[m_j][1-n_j] times
jm, with F = [[jp, jm], [jm, jp]], so in a sector of parity s

    B_s = F (x) F (x) ... (x) F  (jp 1 + s jm C),

a Kronecker product of L^2 - 1 copies of F times a term in C, the map
n -> complement of n in L^2 - 1 bits.  `apply` evaluates T x = W B_s W x
in that form: x times W viewed as a tensor with one axis of length 2 per
bit, F contracted with every axis (tensordot), the C term as the reversed
vector (complementing every bit of an index i gives N - 1 - i), W again.
"""
from __future__ import annotations

import math
from typing import Dict, Tuple

import numpy as np


def couplings(kp: float) -> Tuple[float, float]:
    """(jp, jm) of one site's factor jp 1 + jm sigma^X."""
    ep, em = math.exp(kp), math.exp(-kp)
    return ep / (ep + em), em / (ep + em)


def slice_bond_sum(idx: np.ndarray, L: int, jx, jy) -> np.ndarray:
    """Bsp of the slice states with the given indices (bit j <=> S_j = -1),
    summed bond by bond from the definition."""
    jx = np.asarray(jx, dtype=np.int64).reshape(L, L)  # [x2][x1]
    jy = np.asarray(jy, dtype=np.int64).reshape(L, L)
    idx = np.asarray(idx, dtype=np.int64)
    B = np.zeros(idx.shape, dtype=np.int64)

    def spin(x1, x2):
        return 1 - 2 * ((idx >> (x1 + L * x2)) & 1)

    for x2 in range(L):
        for x1 in range(L):
            s = spin(x1, x2)
            B += jx[x2, x1] * s * spin((x1 + 1) % L, x2)
            B += jy[x2, x1] * s * spin(x1, (x2 + 1) % L)
    return B


def sector_dim(L: int) -> int:
    return 1 << (L * L - 1)


def weights(L: int, k: float, jx, jy) -> np.ndarray:
    """Diagonal of W on the sector basis: exp(k Bsp(n) / 2), n < 2^(L^2-1)."""
    B = slice_bond_sum(np.arange(sector_dim(L), dtype=np.int64), L, jx, jy)
    return np.exp(0.5 * k * B.astype(np.float64))


def apply(L: int, k: float, kp: float, jx, jy, parity: int, x: np.ndarray,
          w: np.ndarray | None = None) -> np.ndarray:
    """T x in the sector of the given parity (+1 even, -1 odd), float64."""
    assert parity in (1, -1)
    n = L * L - 1
    N = 1 << n
    x = np.asarray(x, dtype=np.float64)
    assert x.shape == (N,)
    if w is None:
        w = weights(L, k, jx, jy)
    jp, jm = couplings(kp)
    F = np.array([[jp, jm], [jm, jp]])
    t = (w * x).reshape((2,) * n)
    for axis in range(n):  # F on every bit (F is symmetric, the order is free)
        t = np.moveaxis(np.tensordot(F, t, axes=([1], [axis])), 0, axis)
    y = t.reshape(N)
    y = jp * y + parity * jm * y[::-1]
    return w * y


def sector_matrix(L: int, k: float, kp: float, jx, jy, parity: int) -> np.ndarray:
    """Dense sector matrix, column by column from `apply` (small L only)."""
    N = sector_dim(L)
    assert N <= 4096
    w = weights(L, k, jx, jy)
    cols = [apply(L, k, kp, jx, jy, parity, e, w) for e in np.eye(N)]
    return np.array(cols).T


def full_matrix(L: int, k: float, kp: float, jx, jy) -> np.ndarray:
    """T on all 2^(L^2) slice states, from its matrix elements (small L only):
    e^{k Bsp(S)/2} prod_j (jp if S_j = S'_j else jm) e^{k Bsp(S')/2}."""
    V = L * L
    assert V <= 12
    idx = np.arange(1 << V, dtype=np.int64)
    w = np.exp(0.5 * k * slice_bond_sum(idx, L, jx, jy).astype(np.float64))
    jp, jm = couplings(kp)
    diff = idx[:, None] ^ idx[None, :]
    nd = np.zeros(diff.shape, dtype=np.int64)
    for j in range(V):
        nd += (diff >> j) & 1
    return w[:, None] * (jp ** (V - nd)) * (jm ** nd) * w[None, :]


def leading_eigenpairs(L: int, k: float, kp: float, jx, jy, parity: int,
                       n_eig: int = 2) -> Dict[str, np.ndarray]:
    """The n_eig largest eigenvalues of a sector (descending) and the
    leading eigenvector: dense for L <= 3, ARPACK on `apply` above."""
    N = sector_dim(L)
    if N <= 4096:
        vals, vecs = np.linalg.eigh(sector_matrix(L, k, kp, jx, jy, parity))
        order = np.argsort(vals)[::-1]
        return {"values": vals[order[:n_eig]], "vector": vecs[:, order[0]]}
    from scipy.sparse.linalg import LinearOperator, eigsh
    w = weights(L, k, jx, jy)
    op = LinearOperator((N, N), matvec=lambda v: apply(L, k, kp, jx, jy, parity, np.ravel(v), w),
                        dtype=np.float64)
    vals, vecs = eigsh(op, k=n_eig, which="LA", tol=1e-13)
    order = np.argsort(vals)[::-1]
    return {"values": vals[order], "vector": vecs[:, order[0]]}


def abs_bound(L: int, k: float, kp: float, jx, jy, x: np.ndarray,
              w: np.ndarray | None = None) -> np.ndarray:
    """|W| |B| |W| |x| elementwise: the even-sector product of |x| with every
    factor's entries taken by absolute value (all of them are positive for
    kp >= 0, so this is `apply` with parity +1), the scale of the rounding
    error of any evaluation order of T x."""
    assert kp >= 0
    return apply(L, k, kp, jx, jy, 1, np.abs(np.asarray(x, dtype=np.float64)), w)


# --------------------------------------------------------------------------
# Ground-state correlations (App. E, the consistency checks of EDQSG): for a
# sector vector v (the leading eigenvector |GS>), M_xy = <GS| sZ_x sZ_y |GS>,
# R_xyzu = <GS| sZ_x sZ_y sZ_z sZ_u |GS>, and the L_tau -> infinity values
#   Q2 = Tr M^2,  F = Tr M Mt,  Q4 = sum_{x,y,z,u} R_xyzu^2,
# Mt_xy = M_xy [cos(2 pi (x1 - y1)/L) + cos(2 pi (x2 - y2)/L)] / 2.
# In either sector the weight of the basis pair {n, ~n} is v_n^2 (the
# operators are even under the global flip), normalised by |v|^2.
# --------------------------------------------------------------------------
def ground_correlations(L: int, v: np.ndarray) -> Dict[str, float]:
    """Q2, Q4, F from the definitions: every ordered pair and quadruple of
    sites summed over every basis state (small L only)."""
    V = L * L
    N = sector_dim(L)
    assert N <= 1 << 8
    p = np.asarray(v, dtype=np.float64) ** 2
    p = p / p.sum()
    idx = np.arange(N, dtype=np.int64)
    S = 1 - 2 * ((idx[:, None] >> np.arange(V)[None, :]) & 1)     # last site +1
    M = np.einsum("n,nx,ny->xy", p, S, S)
    x1 = np.arange(V) % L
    x2 = np.arange(V) // L
    cw = 0.5 * (np.cos(2 * math.pi * (x1[:, None] - x1[None, :]) / L) +
                np.cos(2 * math.pi * (x2[:, None] - x2[None, :]) / L))
    Mt = M * cw
    Q4 = 0.0
    for x in range(V):
        for y in range(V):
            Sxy = p * S[:, x] * S[:, y]
            R = np.einsum("n,nz,nu->zu", Sxy, S, S)
            Q4 += float((R ** 2).sum())
    return {"Q2": float(np.trace(M @ M)), "Q4": Q4, "F": float(np.trace(M @ Mt))}


def walsh_hadamard(x: np.ndarray) -> np.ndarray:
    """sum_n x_n (-1)^popcount(n & m) for every mask m, one XOR-stride round
    per bit (the unnormalised Walsh-Hadamard transform)."""
    x = np.asarray(x, dtype=np.float64)
    N = x.size
    n = N.bit_length() - 1
    idx = np.arange(N, dtype=np.int64)
    for j in range(n):
        sign = 1 - 2 * ((idx >> j) & 1)
        x = sign * x + x[idx ^ (1 << j)]
    return x


def ground_correlations_wht(L: int, v: np.ndarray) -> Dict[str, float]:
    """The same three numbers from the Walsh-Hadamard transform W of v^2:
    for a set S of sites, R_S = W[S without the last site] / W[0] (the last
    site's spin is +1 in the sector states).  Ordered pairs and quadruples
    of sites reduce to the set of sites met an odd number of times, which is
    empty, a pair or a quadruple:
      Q2 = V + 2 sum_{|S|=2} R_S^2,
      F  = V + sum_{S={x,y}} R_S^2 [cos(2 pi dx1/L) + cos(2 pi dx2/L)],
      Q4 = 3V^2 - 2V + (12V - 16) sum_{|S|=2} R_S^2 + 24 sum_{|S|=4} R_S^2."""
    from itertools import combinations
    V = L * L
    W = walsh_hadamard(np.asarray(v, dtype=np.float64) ** 2)
    W = W / W[0]
    last = V - 1

    def mask(s):
        return sum(1 << i for i in s if i != last)

    s2 = sF = 0.0
    for x, y in combinations(range(V), 2):
        r2 = W[mask((x, y))] ** 2
        s2 += r2
        sF += r2 * (math.cos(2 * math.pi * (x % L - y % L) / L) +
                    math.cos(2 * math.pi * (x // L - y // L) / L))
    s4 = sum(W[mask(q)] ** 2 for q in combinations(range(V), 4))
    return {"Q2": V + 2 * s2, "Q4": 3 * V * V - 2 * V + (12 * V - 16) * s2 + 24 * s4,
            "F": V + sF}


def xi2(Q2: float, F: float, L: int) -> float:
    """Second-moment correlation length (App. E): sqrt(Q2/F - 1) / (2 sin(pi/L))."""
    return math.sqrt(Q2 / F - 1.0) / (2.0 * math.sin(math.pi / L))


def odd_weight(lam_even: float, lam_odd: float, L_tau: int) -> float:
    """Weight of the odd sector's leading state in a periodic prism of L_tau
    slices when only the two leading states are kept: lambda_o^L_tau /
    (lambda_e^L_tau + lambda_o^L_tau); L_tau = 0 stands for infinity."""
    if L_tau == 0:
        return 0.0
    x = L_tau * math.log(lam_even / lam_odd)
    if x > 0:  # the same ratio written so that a long prism does not overflow
        return math.exp(-x) / (1.0 + math.exp(-x))
    return 1.0 / (1.0 + math.exp(x))


def correlations_mixed(L: int, v_even: np.ndarray, v_odd: np.ndarray, w: float) -> Dict[str, float]:
    """Q2, Q4, F of the mixture (1 - w) |e><e| + w |o><o| of two unit-weight
    sector states (App. E, the finite-L_tau estimates of EDQSG): M and R are
    linear in the state's weights, so they mix, and Q2, Q4, F follow from the
    mixed correlations as for one state (Walsh-Hadamard route)."""
    from itertools import combinations
    V = L * L
    pe = np.asarray(v_even, dtype=np.float64) ** 2
    po = np.asarray(v_odd, dtype=np.float64) ** 2
    p = (1.0 - w) * pe / pe.sum() + w * po / po.sum()
    Wt = walsh_hadamard(p)
    Wt = Wt / Wt[0]
    last = V - 1

    def mask(s):
        return sum(1 << i for i in s if i != last)

    s2 = sF = 0.0
    for x, y in combinations(range(V), 2):
        r2 = Wt[mask((x, y))] ** 2
        s2 += r2
        sF += r2 * (math.cos(2 * math.pi * (x % L - y % L) / L) +
                    math.cos(2 * math.pi * (x // L - y // L) / L))
    s4 = sum(Wt[mask(q)] ** 2 for q in combinations(range(V), 4))
    return {"Q2": V + 2 * s2, "Q4": 3 * V * V - 2 * V + (12 * V - 16) * s2 + 24 * s4,
            "F": V + sF}
