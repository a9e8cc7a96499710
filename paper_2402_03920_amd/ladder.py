"""Learned Gamma ladders for parallel tempering.

A small MLP (kernels in csrc/qsg_mlp.hip, reached through the C ABI) maps a
sample's features to a 32-point ladder meant to equalise the exchange
acceptance between neighbouring slots; the fixed geometric ladder is both
the fallback (when the predicted acceptance is below a floor) and the
yardstick.  Training targets come from the acceptance measured in plain
runs of the same library.

Host-side code here only prepares inputs (features, targets) and moves
buffers; forward, backward, loss, Adam and the ladder decode run on the GPU.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Sequence, Tuple

import numpy as np

from . import qsg

N_POINTS = 32
N_INC = N_POINTS - 1
BARRIER_FLOOR = 1e-3
RHO_FLOOR = 1e-4


# ------------------------------------------------------------- features
def frustrated_fraction(jx: np.ndarray, jy: np.ndarray, L: int, lane: int = 0) -> float:
    """Fraction of plaquettes whose four couplings multiply to -1 (lane's
    sample).  Plaquette (x, y): Jx(x,y), Jy(x+1,y), Jx(x,y+1), Jy(x,y)."""
    bx = ((np.asarray(jx, np.uint64) >> np.uint64(lane)) & np.uint64(1)).astype(np.int64).reshape(L, L)
    by = ((np.asarray(jy, np.uint64) >> np.uint64(lane)) & np.uint64(1)).astype(np.int64).reshape(L, L)
    s = bx + np.roll(by, -1, axis=1) + np.roll(bx, -1, axis=0) + by  # [y][x]
    return float(np.mean(s % 2))


def features(L, L_tau, beta, ffrac, gmin, gmax) -> np.ndarray:
    """Network input: (L, L_tau, beta, frustrated fraction, Gamma_min,
    Gamma_max), scaled to order one."""
    return np.array([L / 16.0, math.log2(L_tau) / 8.0, math.log(beta) / 4.0,
                     (ffrac - 0.5) * 4.0, math.log(gmin), math.log(gmax)], dtype=np.float32)


# -------------------------------------------------------------- targets
def targets_from_acceptance(gammas: Sequence[float], acc_rate: Sequence[float]
                            ) -> Tuple[np.ndarray, float]:
    """Ladder that equalises the exchange barrier, as 31 increments of
    log Gamma summing to one, and the log of the total barrier.

    The barrier accumulated along the measured ladder is the running sum of
    the rejection rates of its gaps, taken as piecewise linear in log Gamma;
    the target ladder puts its 32 points at equal fractions of the total."""
    x = np.log(np.asarray(gammas, dtype=np.float64))
    rho = np.maximum(1.0 - np.asarray(acc_rate, dtype=np.float64), RHO_FLOOR)
    lam = np.concatenate([[0.0], np.cumsum(rho)])
    total = float(lam[-1])
    lev = total * np.arange(N_POINTS) / N_INC
    xs = np.interp(lev, lam, x)
    xs[0], xs[-1] = x[0], x[-1]
    inc = np.diff(xs) / (x[-1] - x[0])
    inc = np.maximum(inc, 0.0)
    inc /= inc.sum()
    return inc.astype(np.float32), float(math.log(max(total, BARRIER_FLOOR)))


def geometric(gmin, gmax, n=N_POINTS) -> np.ndarray:
    g = np.arange(n, dtype=np.float64)
    lad = gmin * (gmax / gmin) ** (g / (n - 1))
    lad[0], lad[-1] = gmin, gmax
    return np.maximum.accumulate(lad)


# ---------------------------------------------------------------- model
class LadderMLP:
    """Parameters and optimiser state on the GPU; every numeric step runs in
    the library's kernels."""

    def __init__(self, seed: int = 0, bf16: bool = True, params: np.ndarray | None = None):
        import torch
        self.torch = torch
        n = int(qsg.lib().qsg_mlp_param_count())
        self.n_params = n
        if params is None:
            params = init_params(seed)
        self.params = torch.tensor(np.asarray(params, np.float32), device="cuda")
        self.bf16 = torch.zeros(n, dtype=torch.int16, device="cuda") if bf16 else None
        self.m = torch.zeros(n, dtype=torch.float32, device="cuda")
        self.v = torch.zeros(n, dtype=torch.float32, device="cuda")
        self.grads = torch.zeros(n, dtype=torch.float32, device="cuda")
        self.step = 0
        if self.bf16 is not None:
            qsg.qsg_mlp_to_bf16(self.params, self.bf16)

    def forward(self, x):
        torch = self.torch
        B = x.shape[0]
        ws = torch.empty(int(qsg.lib().qsg_mlp_workspace_floats(B)), dtype=torch.float32,
                         device="cuda")
        out = torch.empty((B, N_POINTS), dtype=torch.float32, device="cuda")
        qsg.qsg_mlp_forward(self.params, self.bf16, x, out, ws)
        return out, ws

    def train_step(self, x, t_inc, t_logL, lr: float) -> "torch.Tensor":
        torch = self.torch
        out, ws = self.forward(x)
        B = x.shape[0]
        dz = torch.empty_like(out)
        loss = torch.empty(B, dtype=torch.float32, device="cuda")
        qsg.qsg_mlp_loss(out, t_inc, t_logL, dz, loss)
        scratch = torch.empty(2 * B * 128, dtype=torch.float32, device="cuda")
        qsg.qsg_mlp_backward(self.params, self.bf16, x, ws, dz, self.grads, scratch)
        self.step += 1
        qsg.qsg_mlp_adam(self.params, self.bf16, self.grads, self.m, self.v, self.step, lr)
        return loss

    def fit(self, X: np.ndarray, T: np.ndarray, logL: np.ndarray, steps: int = 2000,
            lr: float = 1e-3, log_every: int = 0) -> List[float]:
        torch = self.torch
        x = torch.tensor(np.asarray(X, np.float32), device="cuda")
        t = torch.tensor(np.asarray(T, np.float32), device="cuda")
        l = torch.tensor(np.asarray(logL, np.float32), device="cuda")
        hist = []
        for i in range(steps):
            loss = self.train_step(x, t, l, lr)
            if log_every and (i % log_every == 0 or i == steps - 1):
                hist.append(float(loss.mean().item()))
        return hist

    def predict(self, X: np.ndarray, gmin: Sequence[float], gmax: Sequence[float]):
        """(ladders [B][32] float64, predicted acceptance [B])."""
        torch = self.torch
        x = torch.tensor(np.asarray(X, np.float32), device="cuda")
        out, _ = self.forward(x)
        B = x.shape[0]
        lo = torch.tensor(np.asarray(gmin, np.float64), device="cuda")
        hi = torch.tensor(np.asarray(gmax, np.float64), device="cuda")
        lad = torch.empty((B, N_POINTS), dtype=torch.float64, device="cuda")
        acc = torch.empty(B, dtype=torch.float32, device="cuda")
        qsg.qsg_mlp_decode(out, lo, hi, lad, acc)
        torch.cuda.synchronize()
        return lad.cpu().numpy(), acc.cpu().numpy()

    def params_numpy(self) -> np.ndarray:
        return self.params.detach().cpu().numpy().astype(np.float64)


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal weights, zero biases, with the output layer scaled down so
    an untrained network starts close to the geometric ladder."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = [(6, 128), (128, 128), (128, 128), (128, 32)]
    parts = []
    for i, (k, n) in enumerate(sizes):
        scale = math.sqrt(2.0 / k) * (0.1 if i == len(sizes) - 1 else 1.0)
        parts.append(rng.normal(0.0, scale, size=k * n))
        parts.append(np.zeros(n))
    return np.concatenate(parts).astype(np.float32)


def choose(ladders: np.ndarray, acc_pred: np.ndarray, gmin, gmax, floor: float = 0.2):
    """Learned ladder where the predicted acceptance reaches the floor,
    geometric ladder otherwise.  Returns (ladders, used_learned mask)."""
    out = np.empty_like(ladders)
    used = np.asarray(acc_pred) >= floor
    for i in range(ladders.shape[0]):
        out[i] = ladders[i] if used[i] else geometric(gmin[i], gmax[i])
    return out, used


@dataclass
class RunStats:
    acc_rate: List[np.ndarray]      # per group, per pair
    rt_count: np.ndarray            # per group: completed round trips, all lanes
    rt_time: np.ndarray             # per group: mean round-trip time (PT steps), nan if none
    pt_steps: int
    wall_s: float


def run_and_measure(groups, sweeps: int, pt_every: int = 10, flags=None) -> RunStats:
    """Run groups from random spins for `sweeps` sweeps and collect exchange
    acceptance and round trips."""
    import time
    import torch
    if flags is None:
        flags = qsg.QSG_BATCHED | qsg.QSG_GRAPH
    with qsg.Ensemble(groups, pt_every=pt_every, swaplog_cap=8) as ens:
        ens.init_spins()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ens.sweep(sweeps, flags)
        ens.sync()
        wall = time.perf_counter() - t0
        _, p = ens.counters()
        acc = ens.accepts()
        rts = ens.roundtrips()
    rates = [a.astype(np.float64) / (64.0 * max(p, 1)) for a in acc]
    cnt = np.array([int(r["count"].sum()) for r in rts])
    tot = np.array([float(r["sum"].sum()) for r in rts])
    with np.errstate(invalid="ignore", divide="ignore"):
        mean_t = np.where(cnt > 0, tot / np.maximum(cnt, 1), np.nan)
    return RunStats(rates, cnt, mean_t, p, wall)
