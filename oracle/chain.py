"""ctypes driver of the plain C chain in qsg_oracle.c (test oracle).

One `OracleGroup` holds the complete state of one group (64 lanes sharing
shape, beta, ladder and Monte Carlo key) in numpy arrays and advances it one
spin at a time through the C code.  See qsg_oracle.c for the conventions.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

from . import tables

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqsg_oracle.so")

_lib: Optional[C.CDLL] = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build
            build.build()
        _lib = C.CDLL(LIB_PATH)
        _lib.oracle_run.restype = C.c_int
        _lib.oracle_run.argtypes = [C.c_void_p, C.c_uint64, C.c_uint32, C.c_int]
        _lib.oracle_pt_step.restype = C.c_int
        _lib.oracle_pt_step.argtypes = [C.c_void_p]
        _lib.oracle_state_size.restype = C.c_size_t
        _lib.oracle_pt_r.restype = C.c_uint32
        _lib.oracle_pt_r.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32,
                                     C.c_uint32, C.c_uint32]
        _lib.oracle_metropolis_r.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32,
                                             C.c_uint32, C.c_uint32, C.c_void_p]
        _lib.oracle_philox4x32_10.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        _lib.oracle_init_couplings.argtypes = [C.c_int, C.c_void_p, C.c_void_p,
                                               C.c_void_p]
        _lib.oracle_init_spins.argtypes = [C.c_int, C.c_int, C.c_int, C.c_uint32,
                                           C.c_uint64, C.c_uint32, C.c_void_p]
        _lib.oracle_site_classes.argtypes = [C.c_int, C.c_int, C.c_int, C.c_void_p,
                                             C.c_void_p, C.c_void_p, C.c_int64,
                                             C.c_int, C.c_void_p, C.c_void_p]
        _lib.oracle_recompute.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p,
                                          C.c_void_p, C.c_void_p, C.c_void_p,
                                          C.c_void_p, C.c_void_p]
    return _lib


def _p(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def metropolis_r(seed, group_id, s, t, g) -> np.ndarray:
    r = np.zeros(64, dtype=np.uint32)
    lib().oracle_metropolis_r(seed, group_id, s, t, g, _p(r))
    return r


def pt_r(seed, group_id, p, g, j) -> int:
    return int(lib().oracle_pt_r(seed, group_id, p, g, j))


def couplings(L: int, j_seeds) -> tuple:
    seeds = np.ascontiguousarray(np.asarray(j_seeds, dtype=np.uint64))
    assert seeds.shape == (64,)
    Jx = np.zeros(L * L, dtype=np.uint64)
    Jy = np.zeros(L * L, dtype=np.uint64)
    lib().oracle_init_couplings(L, _p(seeds), _p(Jx), _p(Jy))
    return Jx, Jy


def initial_spins(L, L_tau, N, group_id, seed, slot_base=0) -> np.ndarray:
    S = np.zeros(N * L_tau * L * L, dtype=np.uint64)
    lib().oracle_init_spins(L, L_tau, N, group_id, seed, slot_base, _p(S))
    return S


def site_classes(L, L_tau, Jx, Jy, cfgs: np.ndarray, lane: int = 0, antiperiodic=False):
    cfgs = np.ascontiguousarray(cfgs, dtype=np.uint64)
    V = L * L * L_tau
    n = cfgs.size // V
    ns = np.zeros(n * V, dtype=np.uint8)
    nt = np.zeros(n * V, dtype=np.uint8)
    lib().oracle_site_classes(L, L_tau, int(bool(antiperiodic)), _p(Jx), _p(Jy), _p(cfgs), n,
                              lane, _p(ns), _p(nt))
    return ns.reshape(n, V), nt.reshape(n, V)


class _State(C.Structure):
    _fields_ = [
        ("L", C.c_int32), ("Ltau", C.c_int32), ("N", C.c_int32),
        ("group_id", C.c_uint32), ("mc_seed", C.c_uint64),
        ("thr", C.c_void_p), ("pt_equal", C.c_void_p), ("sw_len", C.c_void_p),
        ("sw_off", C.c_void_p), ("sw_thr", C.c_void_p),
        ("Jx", C.c_void_p), ("Jy", C.c_void_p), ("spins", C.c_void_p),
        ("Bsp", C.c_void_p), ("Bt", C.c_void_p), ("walker", C.c_void_p),
        ("rt_state", C.c_void_p), ("rt_tlast", C.c_void_p),
        ("rt_count", C.c_void_p), ("rt_sum", C.c_void_p), ("acc", C.c_void_p),
        ("swaplog", C.c_void_p), ("log_cap", C.c_uint64),
        ("sum_Bsp", C.c_void_p), ("sum_Bt", C.c_void_p), ("sum_q", C.c_void_p),
        ("sum_q2", C.c_void_p), ("counters", C.c_void_p), ("hist", C.c_void_p),
        ("slot_base", C.c_uint32), ("tau_anti", C.c_uint32), ("exch_all", C.c_uint32),
    ]


class OracleGroup:
    """Full state of one group, advanced by the C oracle.

    thr / swap tables come from `oracle.tables` (mpmath) unless given, so
    the tests can also drive the chain with hand-made tables.
    """

    def __init__(self, L, L_tau, beta, gammas, group_id, mc_seed, j_seeds,
                 log_cap=4096, thr=None, swap=None, spins=None, slot_base=0,
                 ladder="gamma", antiperiodic=False):
        """`gammas` is the ladder: transverse fields (ascending) for
        ladder="gamma", couplings k_g (descending) for ladder="k".
        antiperiodic: S(tau + L_tau) = -S(tau) instead of periodic in tau."""
        self.antiperiodic = bool(antiperiodic)
        if ladder not in ("gamma", "k"):
            raise ValueError("ladder must be 'gamma' or 'k'")
        self.ladder = ladder
        self.L, self.L_tau, self.beta = int(L), int(L_tau), float(beta)
        self.gammas = np.asarray(gammas, dtype=np.float64)
        self.N = len(self.gammas)
        self.group_id, self.mc_seed = int(group_id), int(mc_seed)
        self.j_seeds = [int(s) for s in j_seeds]
        N, V = self.N, self.L * self.L * self.L_tau
        self.V = V
        if thr is None:
            thr = (tables.metropolis_thresholds_k(self.gammas) if ladder == "k"
                   else tables.metropolis_thresholds(beta, L_tau, self.gammas))
        self.thr = np.ascontiguousarray(thr, dtype=np.uint32).reshape(N, 15)
        if swap is None:
            swap = (tables.flat_swap_tables_k(self.gammas) if ladder == "k"
                    else tables.flat_swap_tables(beta, L_tau, self.gammas))
        eq, ln, off, flat = swap
        self.pt_equal = np.ascontiguousarray(eq, dtype=np.uint8)
        self.sw_len = np.ascontiguousarray(ln, dtype=np.uint32)
        self.sw_off = np.ascontiguousarray(off, dtype=np.uint64)
        self.sw_thr = np.ascontiguousarray(flat, dtype=np.uint32)
        if self.pt_equal.size == 0:  # N == 1 is never used by the chain
            self.pt_equal = np.zeros(1, np.uint8)
            self.sw_len = np.zeros(1, np.uint32)
            self.sw_off = np.zeros(1, np.uint64)
        self.Jx, self.Jy = couplings(self.L, self.j_seeds)
        self.slot_base = int(slot_base)
        self.spins = (initial_spins(self.L, self.L_tau, N, self.group_id,
                                    self.mc_seed, self.slot_base) if spins is None
                      else np.ascontiguousarray(spins, dtype=np.uint64).copy())
        self.Bsp = np.zeros(N * 64, dtype=np.int32)
        self.Bt = np.zeros(N * 64, dtype=np.int32)
        q = np.zeros(N * 32, dtype=np.int64)
        lib().oracle_recompute(self.L, self.L_tau, int(self.antiperiodic), N, _p(self.Jx), _p(self.Jy),
                               _p(self.spins), _p(self.Bsp), _p(self.Bt), _p(q))
        self.walker = np.repeat(np.arange(N, dtype=np.uint8), 64)
        self.rt_state = np.zeros(N * 64, dtype=np.uint8)
        self.rt_state[0:64] = 1  # walker 0 starts at slot 0
        self.rt_tlast = np.zeros(N * 64, dtype=np.uint32)
        self.rt_count = np.zeros(N * 64, dtype=np.uint32)
        self.rt_sum = np.zeros(N * 64, dtype=np.uint64)
        self.acc = np.zeros(max(N - 1, 1), dtype=np.uint64)
        self.log_cap = int(log_cap)
        self.swaplog = np.zeros(self.log_cap * max(N - 1, 1), dtype=np.uint64)
        self.sum_Bsp = np.zeros(N * 64, dtype=np.int64)
        self.sum_Bt = np.zeros(N * 64, dtype=np.int64)
        self.sum_q = np.zeros(N * 32, dtype=np.int64)
        self.sum_q2 = np.zeros(N * 32, dtype=np.int64)
        self.counters = np.zeros(2, dtype=np.uint64)
        self.hist = np.zeros(N * 1024, dtype=np.uint32)
        self._st = _State(
            self.L, self.L_tau, N, self.group_id, self.mc_seed,
            _p(self.thr), _p(self.pt_equal), _p(self.sw_len), _p(self.sw_off),
            _p(self.sw_thr), _p(self.Jx), _p(self.Jy), _p(self.spins),
            _p(self.Bsp), _p(self.Bt), _p(self.walker), _p(self.rt_state),
            _p(self.rt_tlast), _p(self.rt_count), _p(self.rt_sum), _p(self.acc),
            _p(self.swaplog), self.log_cap, _p(self.sum_Bsp), _p(self.sum_Bt),
            _p(self.sum_q), _p(self.sum_q2), _p(self.counters), _p(self.hist), self.slot_base,
            int(self.antiperiodic), 1 if ladder == "k" else 0)

    @classmethod
    def from_workload_group(cls, grp, **kw):
        return cls(grp.L, grp.L_tau, grp.beta, grp.gammas, grp.group_id,
                   grp.mc_seed, grp.j_seeds, ladder=grp.ladder,
                   antiperiodic=grp.antiperiodic, **kw)

    @classmethod
    def single_slot(cls, grp, g, **kw):
        """Slot g of a group on its own (valid between PT steps, where the
        slots of a group evolve independently)."""
        return cls(grp.L, grp.L_tau, grp.beta, [grp.gammas[g]], grp.group_id,
                   grp.mc_seed, grp.j_seeds, slot_base=g, ladder=grp.ladder,
                   antiperiodic=grp.antiperiodic, **kw)

    # ------------------------------------------------------------------
    @property
    def t(self) -> int:
        return int(self.counters[0])

    @property
    def p(self) -> int:
        return int(self.counters[1])

    def run(self, n_sweeps: int, pt_every: int = 10, threads: int = 0) -> None:
        rc = lib().oracle_run(C.addressof(self._st), int(n_sweeps),
                              int(pt_every), int(threads))
        if rc != 0:
            raise AssertionError("oracle: tracked bond sums differ from recomputed")

    def pt_step(self) -> None:
        if lib().oracle_pt_step(C.addressof(self._st)) != 0:
            raise AssertionError("oracle: tracked bond sums differ from recomputed")

    def recompute(self):
        N = self.N
        Bsp = np.zeros(N * 64, dtype=np.int32)
        Bt = np.zeros(N * 64, dtype=np.int32)
        q = np.zeros(N * 32, dtype=np.int64)
        lib().oracle_recompute(self.L, self.L_tau, int(self.antiperiodic), N, _p(self.Jx), _p(self.Jy),
                               _p(self.spins), _p(Bsp), _p(Bt), _p(q))
        return Bsp.reshape(N, 64), Bt.reshape(N, 64), q.reshape(N, 32)

    def spins_array(self) -> np.ndarray:
        return self.spins.reshape(self.N, self.L_tau, self.L, self.L)

    def swaplog_rows(self) -> np.ndarray:
        """Swap masks of the PT steps done so far (oldest first, ring order)."""
        n = min(self.p, self.log_cap)
        rows = self.swaplog.reshape(self.log_cap, max(self.N - 1, 1))
        idx = [(self.p - n + i) % self.log_cap for i in range(n)]
        return rows[idx].copy()
