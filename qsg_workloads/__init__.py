"""Seeded synthetic inputs shared by the oracle and the GPU path.

This module only *describes* workloads: lattice shapes, inverse temperature,
transverse-field ladders as IEEE doubles, seeds.  It holds none of the
method's arithmetic (no couplings, thresholds, random streams or updates):
both sides derive those from these inputs with their own code.

Workloads follow the evaluation set-up of the method: 2D +-J spin glass on an
L x L periodic square lattice, L_tau imaginary-time slices, couplings
J = +-1 i.i.d. with p = 1/2 (paper: Sec. 1, Eq. (1); sample seeds of the
input file, App. A), a ladder of transverse fields for parallel tempering
(Sec. 2.1), and an update schedule of `pt_every` full sweeps per PT step
(App. A, the "ptfr" field).

The transfer-matrix product (Sec. 2.2) takes its couplings and vectors as
plain inputs; `transfer_case` draws them here (numpy PCG64, J = +-1 with
p = 1/2, vector entries standard normal), with the paper's EDQSG example
coupling k = 0.31 in the equal-coupling form as the default.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Sequence

import numpy as np

MC_SEED = 42


def geometric_ladder(gmin: float, gmax: float, n: int) -> np.ndarray:
    """Gamma_g = gmin * (gmax/gmin)**(g/(n-1)), g = 0..n-1, ascending doubles.

    Generated once here (numpy float64) and handed as doubles to both the
    oracle and the library, so the two never disagree over libm rounding.
    """
    if n < 1:
        raise ValueError("a ladder needs at least one point")
    if n == 1:
        return np.array([float(gmin)])
    g = np.arange(n, dtype=np.float64)
    lad = gmin * (gmax / gmin) ** (g / (n - 1))
    lad[0] = gmin
    lad[-1] = gmax
    return np.maximum.accumulate(lad)


@dataclass
class Group:
    """One group: 64 bit-lanes that share shape, beta, ladder and MC key.

    j_seeds has 64 entries (one per lane).  All equal means one disorder
    sample with 64 replicas; distinct values put a different sample in
    every lane.  `gammas` is the ladder: transverse fields, ascending, for
    ladder == "gamma"; couplings k_g, descending, for ladder == "k" (the
    paper's own PT variable; beta is then unused).
    """

    L: int
    L_tau: int
    beta: float
    gammas: np.ndarray
    group_id: int
    mc_seed: int
    j_seeds: List[int]
    ladder: str = "gamma"
    antiperiodic: bool = False  # S(tau + L_tau) = -S(tau) (else periodic in tau)

    @property
    def n_gamma(self) -> int:
        return int(len(self.gammas))

    @property
    def words(self) -> int:
        return self.n_gamma * self.L_tau * self.L * self.L

    @property
    def spin_updates_per_sweep(self) -> int:
        return 64 * self.words


@dataclass
class Workload:
    name: str
    groups: List[Group]
    sweeps: int
    pt_every: int = 10
    notes: str = ""

    def spin_updates_per_sweep(self) -> int:
        return sum(g.spin_updates_per_sweep for g in self.groups)

    def spin_bytes(self) -> int:
        return 8 * sum(g.words for g in self.groups)


def _replicas(seed: int) -> List[int]:
    return [int(seed)] * 64


def plain_small() -> Workload:
    """One sample, L=8, L_tau=32, beta=4, 16 Gammas geometric in [1.5, 4.5],
    64 replicas in the lanes, 1000 sweeps, PT every 10, J seed 1, MC seed 42."""
    lad = geometric_ladder(1.5, 4.5, 16)
    g = Group(8, 32, 4.0, lad, 0, MC_SEED, _replicas(1))
    return Workload("plain L=8 Ltau=32 NG=16 1 sample", [g], 1000, 10)


def plain_large(n_samples: int = 64) -> Workload:
    """64 samples (one group each, 64 replicas), L=16, L_tau=128, beta=8,
    32 Gammas geometric in [2, 4], J seeds 1..64, 10^4 sweeps, PT every 10."""
    lad = geometric_ladder(2.0, 4.0, 32)
    groups = [Group(16, 128, 8.0, lad, i, MC_SEED, _replicas(i + 1))
              for i in range(n_samples)]
    return Workload("plain L=16 Ltau=128 NG=32 64 samples", groups, 10_000, 10)


def uneven_manifest_rows(n: int = 256, seed: int = 3):
    """Uneven ensemble: L ~ U{8,12,16,20,24}, L_tau ~ U{64,128,256},
    N_Gamma ~ U{24..48}, drawn by numpy PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Ls = rng.choice(np.array([8, 12, 16, 20, 24]), size=n)
    Lts = rng.choice(np.array([64, 128, 256]), size=n)
    NGs = rng.integers(24, 49, size=n)
    return [(int(a), int(b), int(c)) for a, b, c in zip(Ls, Lts, NGs)]


def uneven_ensemble(n_samples: int = 256) -> Workload:
    """256 samples of uneven shape, beta = L_tau/16, Gammas geometric in
    [2, 4], J seeds 1..256, 1000 sweeps, PT every 10."""
    rows = uneven_manifest_rows(256)[:n_samples]
    groups = []
    for i, (L, Lt, ng) in enumerate(rows):
        groups.append(Group(L, Lt, Lt / 16.0, geometric_ladder(2.0, 4.0, ng),
                            i, MC_SEED, _replicas(i + 1)))
    return Workload("batched uneven 256 samples", groups, 1000, 10)


def production() -> Workload:
    """L=24, L_tau=2048, beta=128, 128 samples packed one per lane in two
    groups (J seeds 1..64 and 65..128), 48 Gammas geometric in [2.8, 3.6],
    10^5 sweeps, PT every 10."""
    lad = geometric_ladder(2.8, 3.6, 48)
    groups = [Group(24, 2048, 128.0, lad, gi, MC_SEED,
                    [1 + 64 * gi + j for j in range(64)]) for gi in range(2)]
    return Workload("production L=24 Ltau=2048 NG=48 128 samples", groups,
                    100_000, 10)


def ladder_eval_rows(n: int = 128, seed: int = 5):
    rng = np.random.Generator(np.random.PCG64(seed))
    return [int(x) for x in rng.choice(np.array([12, 16, 20, 24]), size=n)]


def ladder_eval(ladders: Sequence[np.ndarray] | None = None,
            n_samples: int = 128) -> Workload:
    """Fresh samples for the learned-ladder evaluation: L in {12,16,20,24},
    L_tau=256, beta=16, 32 Gammas in [2, 4] (geometric unless `ladders`
    given), J seeds 10001.., 10^4 sweeps, PT every 10."""
    Ls = ladder_eval_rows(128)[:n_samples]
    groups = []
    for i, L in enumerate(Ls):
        lad = geometric_ladder(2.0, 4.0, 32) if ladders is None else np.asarray(
            ladders[i], dtype=np.float64)
        groups.append(Group(L, 256, 16.0, lad, i, MC_SEED, _replicas(10001 + i)))
    return Workload("learned-ladder eval", groups, 10_000, 10)


def linear_k_ladder(kmax: float, kmin: float, n: int) -> np.ndarray:
    """n couplings from kmax down to kmin, equally spaced (descending)."""
    if n == 1:
        return np.array([float(kmax)])
    lad = np.linspace(float(kmax), float(kmin), n)
    lad[0], lad[-1] = kmax, kmin
    return np.minimum.accumulate(lad)


def coupling_ladder(n_samples: int = 64) -> Workload:
    """The paper's own parametrisation (one coupling k on every bond, PT over
    k): 64 samples (64 replicas each), L=16, L_tau=128, 32 couplings from
    0.33 down to 0.25 around the paper's k ~ 0.29, J seeds 1..64, 10^4
    sweeps, PT every 10.  beta is unused by this form (set to 1)."""
    lad = linear_k_ladder(0.33, 0.25, 32)
    groups = [Group(16, 128, 1.0, lad, i, MC_SEED, _replicas(i + 1), ladder="k")
              for i in range(n_samples)]
    return Workload("k ladder L=16 Ltau=128 NK=32 64 samples", groups, 10_000, 10)


def tiny_k_group(L=4, L_tau=8, n_k=3, kmax=0.5, kmin=0.2, group_id=0, mc_seed=MC_SEED,
                 j_seed=1, per_lane=False) -> Group:
    seeds = [j_seed + j for j in range(64)] if per_lane else _replicas(j_seed)
    return Group(L, L_tau, 1.0, linear_k_ladder(kmax, kmin, n_k), group_id, mc_seed, seeds,
                 ladder="k")


def tiny_group(L=4, L_tau=8, beta=1.0, n_gamma=3, gmin=0.5, gmax=2.0,
               group_id=0, mc_seed=MC_SEED, j_seed=1, per_lane=False,
               antiperiodic=False) -> Group:
    lad = geometric_ladder(gmin, gmax, n_gamma)
    seeds = [j_seed + j for j in range(64)] if per_lane else _replicas(j_seed)
    return Group(L, L_tau, beta, lad, group_id, mc_seed, seeds, antiperiodic=antiperiodic)


ALL = {
    "plain-small": plain_small,
    "plain-large": plain_large,
    "uneven": uneven_ensemble,
    "production": production,
    "ladder-eval": ladder_eval,
    "k-ladder": coupling_ladder,
}


@dataclass
class TransferCase:
    L: int
    k: float
    k_perp: float
    jx: np.ndarray   # +-1 per site j = x1 + L x2, bond (j, +x)
    jy: np.ndarray   # +-1 per site, bond (j, +y)
    seed: int

    def vector(self, stream: int = 0) -> np.ndarray:
        """Standard-normal sector vector of 2^(L^2 - 1) doubles."""
        rng = np.random.default_rng([self.seed, 1 + stream])
        return rng.standard_normal(1 << (self.L * self.L - 1))


def transfer_case(L: int = 5, k: float = 0.31, k_perp: float | None = None,
                  seed: int = 6009) -> TransferCase:
    """One disorder sample of an L x L slice for the transfer matrix."""
    rng = np.random.default_rng(seed)
    jx = 1 - 2 * rng.integers(0, 2, L * L)
    jy = 1 - 2 * rng.integers(0, 2, L * L)
    return TransferCase(L, float(k), float(k if k_perp is None else k_perp), jx, jy, seed)
