"""Pins of the transfer-matrix oracle (Sec. 2.2, App. D) against what the
mathematics fixes: the matrix elements in the full spin basis, the partition
function of the Trotter-Suzuki prism by exact enumeration, closed forms at
J = 0 and at a large time coupling, symmetry.  None compares the sector
product with itself."""
import math

import numpy as np
import pytest

from oracle import exact, transfer


def random_j(L, seed):
    rng = np.random.default_rng(seed)
    return (1 - 2 * rng.integers(0, 2, L * L)), (1 - 2 * rng.integers(0, 2, L * L))


def sector_basis(L, parity):
    """Columns (|n> + parity |~n>)/sqrt(2) in the full 2^(L^2) basis."""
    V = L * L
    N = 1 << (V - 1)
    U = np.zeros((1 << V, N))
    for n in range(N):
        U[n, n] += 1 / math.sqrt(2)
        U[((1 << V) - 1) ^ n, n] += parity / math.sqrt(2)
    return U


@pytest.mark.parametrize("L,seed", [(2, 1), (3, 2)])
def test_sectors_are_the_full_matrix_in_the_parity_basis(L, seed):
    """The sector product (W, XOR-stride rounds, the complement round with
    the sector's sign, W) equals U^T T U with T built element by element on
    all 2^(L^2) states and U the parity basis of App. D."""
    jx, jy = random_j(L, seed)
    k, kp = 0.31, 0.27
    T = transfer.full_matrix(L, k, kp, jx, jy)
    assert np.allclose(T, T.T, rtol=0, atol=1e-15 * np.abs(T).max())
    for parity in (1, -1):
        U = sector_basis(L, parity)
        want = U.T @ T @ U
        got = transfer.sector_matrix(L, k, kp, jx, jy, parity)
        assert np.allclose(got, want, rtol=1e-12, atol=1e-14 * np.abs(want).max())
    # parity commutes with T: the two sectors hold the whole spectrum
    ev = np.sort(np.linalg.eigvalsh(T))
    both = np.sort(np.concatenate([np.linalg.eigvalsh(transfer.sector_matrix(L, k, kp, jx, jy, p))
                                   for p in (1, -1)]))
    assert np.allclose(ev, both, rtol=1e-12, atol=1e-13 * ev.max())


@pytest.mark.parametrize("L,L_tau,seed,k,kp", [(2, 4, 3, 0.4, 0.3), (2, 5, 4, 0.25, 0.6),
                                                (3, 2, 5, 0.3, 0.2)])
def test_trace_is_the_prism_partition_function(L, L_tau, seed, k, kp):
    """Z = sum over every configuration of the L x L x L_tau prism of
    exp(k Bsp + kp Bt) (direct enumeration, the chain's weight) equals
    (2 cosh kp)^(L^2 L_tau) Tr T^L_tau, the trace summed over both
    sectors' eigenvalues."""
    jx, jy = random_j(L, seed)
    _, Bsp, Bt = exact.enumerate_states(L, L_tau, jx, jy)
    Z = np.exp(k * Bsp + kp * Bt).sum()
    lam = np.concatenate([np.linalg.eigvalsh(transfer.sector_matrix(L, k, kp, jx, jy, p))
                          for p in (1, -1)])
    tr = (lam ** L_tau).sum() * (2 * math.cosh(kp)) ** (L * L * L_tau)
    assert abs(tr / Z - 1) < 1e-11


@pytest.mark.parametrize("L", [2, 3])
def test_free_spins_closed_form(L):
    """J = 0: T is the product of the site factors, whose eigenvalues are
    1 and tanh kp; the even sector holds products with an even number of
    tanh factors (leading 1, then tanh^2 with multiplicity C(L^2, 2)), the
    odd sector an odd number (leading tanh, L^2 times)."""
    V = L * L
    z = np.zeros(V, dtype=np.int64)
    kp = 0.45
    t = math.tanh(kp)
    ev = np.sort(np.linalg.eigvalsh(transfer.sector_matrix(L, 0.7, kp, z, z, 1)))[::-1]
    od = np.sort(np.linalg.eigvalsh(transfer.sector_matrix(L, 0.7, kp, z, z, -1)))[::-1]
    assert abs(ev[0] - 1) < 1e-14
    assert np.allclose(ev[1:1 + V * (V - 1) // 2], t ** 2, rtol=1e-12)
    assert np.allclose(od[:V], t, rtol=1e-12)
    assert abs(od[V] - t ** 3) < 1e-12
    # the uniform even vector is the leading eigenvector
    one = np.ones(1 << (V - 1))
    assert np.allclose(transfer.apply(L, 0.7, kp, z, z, 1, one), one, rtol=1e-14)


@pytest.mark.parametrize("L,seed", [(2, 6), (3, 7)])
def test_large_time_coupling_is_classical(L, seed):
    """kp large: jm / jp = e^{-2 kp} vanishes, B -> 1 and T -> W^2, so each
    pair {n, ~n} gives one even and one odd eigenvalue exp(k Bsp(n)): the
    spectrum is the classical slice's Boltzmann weights (brute force over
    all states)."""
    jx, jy = random_j(L, seed)
    k = 0.35
    idx = np.arange(1 << (L * L - 1))
    cls = np.sort(np.exp(k * transfer.slice_bond_sum(idx, L, jx, jy).astype(float)))
    for p in (1, -1):
        ev = np.sort(np.linalg.eigvalsh(transfer.sector_matrix(L, k, 25.0, jx, jy, p)))
        assert np.allclose(ev, cls, rtol=1e-12)


def test_bond_sum_matches_the_prism_bond_sum():
    """The slice bond sum is the chain's Bsp of a one-slice prism."""
    L = 3
    jx, jy = random_j(L, 8)
    idx = np.arange(1 << (L * L))
    Bsp, _ = exact.bond_sums(exact.spins_from_index(idx, L * L), L, 1, jx, jy)
    assert np.array_equal(transfer.slice_bond_sum(idx, L, jx, jy), Bsp)


def test_symmetric_and_bounded_at_L4():
    """L = 4 (2^15 per sector): <y, T x> = <T y, x>, and |T x| <= |T| |x|."""
    L = 4
    jx, jy = random_j(L, 9)
    rng = np.random.default_rng(10)
    N = transfer.sector_dim(L)
    x, y = rng.standard_normal(N), rng.standard_normal(N)
    for p in (1, -1):
        Tx = transfer.apply(L, 0.29, 0.29, jx, jy, p, x)
        Ty = transfer.apply(L, 0.29, 0.29, jx, jy, p, y)
        assert abs(y @ Tx - Ty @ x) < 1e-12 * np.abs(y) @ np.abs(Tx)
        assert np.all(np.abs(Tx) <= transfer.abs_bound(L, 0.29, 0.29, jx, jy, x) * (1 + 1e-12))


def test_leading_eigenpairs_at_L4_are_eigenpairs():
    """ARPACK on the sector product: residual |T v - lambda v| tiny, the
    leading even eigenvalue above the leading odd one (ground state even),
    and the even leading vector of one sign (Perron-Frobenius: the even
    sector's matrix has positive entries)."""
    L = 4
    jx, jy = random_j(L, 11)
    k = kp = 0.3
    e = transfer.leading_eigenpairs(L, k, kp, jx, jy, 1)
    o = transfer.leading_eigenpairs(L, k, kp, jx, jy, -1)
    for r, p in ((e, 1), (o, -1)):
        v = r["vector"]
        res = transfer.apply(L, k, kp, jx, jy, p, v) - r["values"][0] * v
        assert np.linalg.norm(res) < 1e-9 * r["values"][0]
    assert e["values"][0] > o["values"][0] > 0
    v = e["vector"] * np.sign(e["vector"].sum())
    assert np.all(v > 0)


def test_walsh_hadamard_is_the_hadamard_matrix():
    from scipy.linalg import hadamard
    rng = np.random.default_rng(12)
    for n in (1, 3, 6):
        x = rng.standard_normal(1 << n)
        assert np.allclose(transfer.walsh_hadamard(x), hadamard(1 << n) @ x, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("L", [2, 3])
def test_ground_correlations_transform_equals_definitions(L):
    """Q2, Q4, F through the Walsh-Hadamard route (the reduction of ordered
    pairs and quadruples to odd-multiplicity sets) equal the plain sums over
    every ordered pair and quadruple of sites: random vectors and the
    leading eigenvector of a sample."""
    rng = np.random.default_rng(13 + L)
    case_j = random_j(L, 14 + L)
    gs = transfer.leading_eigenpairs(L, 0.31, 0.31, *case_j, 1)["vector"]
    for v in (rng.standard_normal(transfer.sector_dim(L)), gs):
        a = transfer.ground_correlations(L, v)
        b = transfer.ground_correlations_wht(L, v)
        for key in ("Q2", "Q4", "F"):
            assert abs(a[key] - b[key]) <= 1e-11 * max(abs(a[key]), 1.0), (key, a, b)


@pytest.mark.parametrize("L", [2, 3, 4])
def test_ground_correlations_closed_forms(L):
    """Independent spins (uniform weights): M = 1, R = 0 off the empty set,
    so Q2 = F = V and Q4 = 3V^2 - 2V; one ordered state: every correlation
    is 1, Q2 = V^2, Q4 = V^4 and F = 0 (the cosines sum to zero)."""
    V = L * L
    N = transfer.sector_dim(L)
    u = transfer.ground_correlations_wht(L, np.ones(N))
    assert np.allclose([u["Q2"], u["Q4"], u["F"]], [V, 3 * V * V - 2 * V, V], rtol=1e-12)
    e = np.zeros(N)
    e[0] = 1.0
    o = transfer.ground_correlations_wht(L, e)
    assert np.allclose([o["Q2"], o["Q4"]], [V * V, V ** 4], rtol=1e-12)
    assert abs(o["F"]) < 1e-9 * V * V


@pytest.mark.parametrize("L", [2, 3])
def test_mixed_correlations(L):
    """The finite-L_tau estimate mixes the two leading states' weights: at
    w = 0 and w = 1 it is the one-state result, and for any w it equals the
    definitions (all ordered pairs and quadruples) evaluated on the mixed
    weights; the odd weight falls off as (lambda_o / lambda_e)^L_tau."""
    rng = np.random.default_rng(40 + L)
    N = transfer.sector_dim(L)
    ve, vo = rng.standard_normal(N), 3.0 * rng.standard_normal(N)
    for key in ("Q2", "Q4", "F"):
        assert abs(transfer.correlations_mixed(L, ve, vo, 0.0)[key] -
                   transfer.ground_correlations_wht(L, ve)[key]) < 1e-9
        assert abs(transfer.correlations_mixed(L, ve, vo, 1.0)[key] -
                   transfer.ground_correlations_wht(L, vo)[key]) < 1e-9
    w = 0.3
    mix = np.sqrt((1 - w) * ve ** 2 / (ve ** 2).sum() + w * vo ** 2 / (vo ** 2).sum())
    a = transfer.correlations_mixed(L, ve, vo, w)
    b = transfer.ground_correlations(L, mix)
    for key in ("Q2", "Q4", "F"):
        assert abs(a[key] - b[key]) < 1e-10 * max(abs(b[key]), 1.0)
    assert transfer.odd_weight(2.0, 1.0, 0) == 0.0
    assert abs(transfer.odd_weight(2.0, 1.0, 3) - 1.0 / 9.0) < 1e-15
    assert abs(transfer.odd_weight(1.0, 1.0, 50) - 0.5) < 1e-15
    assert transfer.odd_weight(2.0, 1.0, 10 ** 9) == 0.0  # long prisms: no overflow
    assert transfer.odd_weight(1.0, 2.0, 10 ** 9) == 1.0
