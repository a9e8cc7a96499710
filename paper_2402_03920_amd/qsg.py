"""Thin ctypes binding of libqsg.so (the C ABI in include/qsg.h).

Argument marshalling only: every step of the hot path runs in the HIP
kernels behind the C ABI.  PyTorch provides the device workspace (a uint8
tensor) and the stream; nothing else.

Functions keep their C names (qsg_create, qsg_sweep, ...).  `Ensemble`
bundles the calls for one set of groups.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libqsg.so")

QSG_OK = 0
QSG_E_INVALID = -1
QSG_E_UNSUPPORTED = -2
QSG_E_DEVICE = -3
QSG_E_STATE = -4
QSG_E_BUFFER = -5
QSG_E_INTERRUPTED = -6

QSG_PLAIN = 0
QSG_BATCHED = 1
QSG_GRAPH = 2
QSG_NO_PT = 4
QSG_FUSED = 8

QSG_M_ENERGY = 1
QSG_M_OVERLAP = 2
QSG_M_ACCEPT = 3
QSG_M_WALKERS = 4
QSG_M_SWAPLOG = 5
QSG_M_ROUNDTRIP = 6
QSG_M_SUMS = 7
QSG_M_COUNTERS = 8
QSG_M_HIST = 9
HIST_BINS = 1024

SUM_STRIDE = 192


class qsg_group_desc(C.Structure):
    _fields_ = [("L", C.c_uint32), ("L_tau", C.c_uint32), ("beta", C.c_double),
                ("n_gamma", C.c_uint32), ("group_id", C.c_uint32),
                ("mc_seed", C.c_uint64), ("j_seed", C.c_uint64 * 64),
                ("swap_table_cap", C.c_uint32), ("ladder_kind", C.c_uint32),
                ("tau_boundary", C.c_uint32), ("reserved", C.c_uint32)]


class qsg_run_config(C.Structure):
    _fields_ = [("pt_every", C.c_uint32), ("swaplog_cap", C.c_uint32),
                ("sweep_split", C.c_uint32), ("tau_tile", C.c_uint32)]


ROUNDTRIP_DTYPE = np.dtype([("state", "<u4"), ("t_last", "<u4"), ("count", "<u4"),
                            ("pad", "<u4"), ("sum", "<u8")])


TM_MAX_L = 5


class qsg_tm_desc(C.Structure):
    _fields_ = [("L", C.c_uint32), ("parity", C.c_int32), ("k", C.c_double),
                ("k_perp", C.c_double), ("jx", C.c_int8 * (TM_MAX_L * TM_MAX_L)),
                ("jy", C.c_int8 * (TM_MAX_L * TM_MAX_L))]


class QSGError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"qsg error {code}: {msg}")
        self.code = code


_lib: Optional[C.CDLL] = None

_SIGS = {
    "qsg_workspace_bytes": (C.c_size_t, [C.c_void_p, C.c_uint32, C.c_void_p]),
    "qsg_create": (C.c_int32, [C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p, C.c_size_t,
                               C.c_void_p, C.POINTER(C.c_void_p)]),
    "qsg_set_gamma_ladder": (C.c_int32, [C.c_void_p, C.c_uint32, C.c_void_p]),
    "qsg_set_k_ladder": (C.c_int32, [C.c_void_p, C.c_uint32, C.c_void_p]),
    "qsg_init_spins": (C.c_int32, [C.c_void_p]),
    "qsg_sweep": (C.c_int32, [C.c_void_p, C.c_uint32, C.c_uint32]),
    "qsg_pt_swap": (C.c_int32, [C.c_void_p]),
    "qsg_measure": (C.c_int32, [C.c_void_p, C.c_uint32, C.c_void_p, C.c_size_t]),
    "qsg_get_spins": (C.c_int32, [C.c_void_p, C.c_uint32, C.c_void_p, C.c_size_t]),
    "qsg_set_spins": (C.c_int32, [C.c_void_p, C.c_uint32, C.c_void_p, C.c_size_t]),
    "qsg_get_couplings": (C.c_int32, [C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p]),
    "qsg_state_bytes": (C.c_size_t, [C.c_void_p]),
    "qsg_get_state": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "qsg_set_state": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "qsg_get_tables": (C.c_int32, [C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_void_p]),
    "qsg_build_tables": (C.c_int32, [C.c_double, C.c_uint32, C.c_uint32, C.c_void_p,
                                     C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p]),
    "qsg_build_tables_k": (C.c_int32, [C.c_uint32, C.c_void_p, C.c_uint32, C.c_void_p,
                                       C.c_void_p, C.c_void_p, C.c_void_p]),
    "qsg_set_deadline": (C.c_int32, [C.c_void_p, C.c_double]),
    "qsg_set_schedule": (C.c_int32, [C.c_void_p, C.c_uint32, C.c_uint32]),
    "qsg_set_colour_schedule": (C.c_int32, [C.c_void_p, C.c_uint32, C.c_uint32, C.c_uint32]),
    "qsg_sync": (C.c_int32, [C.c_void_p]),
    "qsg_last_error": (C.c_char_p, [C.c_void_p]),
    "qsg_destroy": (None, [C.c_void_p]),
    "qsg_philox": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p]),
    "qsg_philox_probe": (C.c_int32, [C.c_uint32, C.c_uint32, C.c_uint64, C.c_void_p, C.c_void_p]),
    "qsg_tau_overlaps": (C.c_int32, [C.c_void_p, C.c_uint32, C.c_uint32, C.c_uint32, C.c_void_p,
                                     C.c_uint32, C.c_void_p, C.c_size_t]),
    "qsg_tau_observables": (C.c_int32, [C.c_void_p, C.c_uint32, C.c_uint32, C.c_uint32,
                                        C.c_uint64, C.c_void_p, C.c_void_p, C.c_void_p]),
    "qsg_tm_dim": (C.c_uint64, [C.c_uint32]),
    "qsg_tm_apply": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "qsg_tm_lanczos_workspace_bytes": (C.c_size_t, [C.c_uint32, C.c_uint32]),
    "qsg_tm_lanczos": (C.c_int32, [C.c_void_p, C.c_uint32, C.c_uint32, C.c_double, C.c_uint64,
                                   C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_void_p]),
    "qsg_tm_correlations_workspace_bytes": (C.c_size_t, [C.c_uint32]),
    "qsg_tm_correlations": (C.c_int32, [C.c_uint32, C.c_void_p, C.c_void_p, C.c_size_t,
                                        C.c_void_p, C.c_void_p]),
    "qsg_tm_correlations_lt_workspace_bytes": (C.c_size_t, [C.c_uint32, C.c_uint32]),
    "qsg_tm_correlations_lt": (C.c_int32, [C.c_uint32, C.c_void_p, C.c_void_p, C.c_double,
                                           C.c_double, C.c_void_p, C.c_uint32, C.c_void_p,
                                           C.c_size_t, C.c_void_p, C.c_void_p]),
    "qsg_mlp_param_count": (C.c_uint32, []),
    "qsg_mlp_workspace_floats": (C.c_size_t, [C.c_uint32]),
    "qsg_mlp_forward_noalloc": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32,
                                            C.c_void_p, C.c_void_p]),
    "qsg_mlp_forward": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32,
                                    C.c_void_p, C.c_void_p, C.c_void_p]),
    "qsg_mlp_backward": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p,
                                     C.c_void_p]),
    "qsg_mlp_loss": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p,
                                 C.c_void_p, C.c_void_p]),
    "qsg_mlp_adam": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_uint32, C.c_float, C.c_void_p]),
    "qsg_mlp_to_bf16": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "qsg_mlp_decode": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p,
                                   C.c_void_p, C.c_void_p]),
}


def lib() -> C.CDLL:
    """Load libqsg.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2402_03920_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def _check(rc: int, ctx=None):
    if rc != QSG_OK:
        msg = lib().qsg_last_error(ctx)
        raise QSGError(rc, msg.decode() if msg else "")


# ------------------------------------------------------------ C-named calls
def qsg_build_tables(beta: float, L_tau: int, gammas: Sequence[float], cap: int = 4096):
    """Host table builder: (thr[N][15], equal[N-1], len[N-1], swap[N-1][cap])."""
    g = np.ascontiguousarray(np.asarray(gammas, dtype=np.float64))
    N = g.size
    pairs = max(N - 1, 1)
    thr = np.zeros(N * 15, np.uint32)
    eq = np.zeros(pairs, np.uint8)
    ln = np.zeros(pairs, np.uint32)
    sw = np.zeros(pairs * cap, np.uint32)
    _check(lib().qsg_build_tables(float(beta), int(L_tau), N, _ptr(g), cap, _ptr(thr),
                                  _ptr(eq), _ptr(ln), _ptr(sw)))
    return thr.reshape(N, 15), eq[:N - 1], ln[:N - 1], sw.reshape(pairs, cap)[:N - 1]


def qsg_build_tables_k(ks: Sequence[float], cap: int = 4096):
    """Host table builder of a coupling ladder, same outputs as qsg_build_tables."""
    k = np.ascontiguousarray(np.asarray(ks, dtype=np.float64))
    N = k.size
    pairs = max(N - 1, 1)
    thr = np.zeros(N * 15, np.uint32)
    eq = np.zeros(pairs, np.uint8)
    ln = np.zeros(pairs, np.uint32)
    sw = np.zeros(pairs * cap, np.uint32)
    _check(lib().qsg_build_tables_k(N, _ptr(k), cap, _ptr(thr), _ptr(eq), _ptr(ln), _ptr(sw)))
    return thr.reshape(N, 15), eq[:N - 1], ln[:N - 1], sw.reshape(pairs, cap)[:N - 1]


LADDER_KINDS = {"gamma": 0, "k": 1}


def make_desc(L, L_tau, beta, n_gamma, group_id, mc_seed, j_seeds,
              swap_table_cap=0, ladder="gamma", antiperiodic=False) -> qsg_group_desc:
    d = qsg_group_desc()
    d.L, d.L_tau, d.beta = int(L), int(L_tau), float(beta)
    d.n_gamma, d.group_id, d.mc_seed = int(n_gamma), int(group_id), int(mc_seed)
    seeds = list(j_seeds)
    if len(seeds) != 64:
        raise ValueError("64 coupling seeds per group")
    for j, s in enumerate(seeds):
        d.j_seed[j] = int(s)
    d.swap_table_cap = int(swap_table_cap)
    d.ladder_kind = LADDER_KINDS[ladder]
    d.tau_boundary = 1 if antiperiodic else 0
    d.reserved = 0
    return d


class Ensemble:
    """A set of groups on the current CUDA (HIP) device and stream.

    `groups` are objects with L, L_tau, beta, gammas, group_id, mc_seed,
    j_seeds and optionally ladder ("gamma" or "k"; e.g. qsg_workloads.Group).
    """

    def __init__(self, groups: Sequence, pt_every: int = 10, swaplog_cap: int = 1024,
                 swap_table_cap: int = 0, stream=None, device=None, sweep_split: int = 0,
                 tau_tile: int = 0):
        import torch  # device memory and streams only
        self._torch = torch
        L_ = lib()
        self.groups = list(groups)
        self.n = len(self.groups)
        self.descs = (qsg_group_desc * self.n)()
        for i, g in enumerate(self.groups):
            self.descs[i] = make_desc(g.L, g.L_tau, g.beta, len(g.gammas), g.group_id,
                                      g.mc_seed, g.j_seeds, swap_table_cap,
                                      getattr(g, "ladder", "gamma"),
                                      getattr(g, "antiperiodic", False))
        self.cfg = qsg_run_config(int(pt_every), int(swaplog_cap), int(sweep_split),
                                  int(tau_tile))
        nbytes = L_.qsg_workspace_bytes(self.descs, self.n, C.byref(self.cfg))
        if nbytes == 0:
            raise QSGError(QSG_E_INVALID, "invalid group description")
        dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        # 256-byte alignment: torch's caching allocator returns >= 512-byte aligned blocks
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        assert self.workspace.data_ptr() % 256 == 0
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        self.ctx = C.c_void_p()
        _check(L_.qsg_create(self.descs, self.n, C.byref(self.cfg),
                             C.c_void_p(self.workspace.data_ptr()), nbytes,
                             C.c_void_p(self.stream.cuda_stream), C.byref(self.ctx)))
        for i, g in enumerate(self.groups):
            if getattr(g, "ladder", "gamma") == "k":
                self.set_k_ladder(i, g.gammas)
            else:
                self.set_gamma_ladder(i, g.gammas)

    # -- lifecycle
    def close(self):
        if self.ctx:
            lib().qsg_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- calls
    def set_gamma_ladder(self, i: int, gammas):
        g = np.ascontiguousarray(np.asarray(gammas, dtype=np.float64))
        if g.size != self.descs[i].n_gamma:
            raise ValueError("ladder length differs from n_gamma")
        _check(lib().qsg_set_gamma_ladder(self.ctx, i, _ptr(g)), self.ctx)

    def set_k_ladder(self, i: int, ks):
        k = np.ascontiguousarray(np.asarray(ks, dtype=np.float64))
        if k.size != self.descs[i].n_gamma:
            raise ValueError("ladder length differs from n_gamma")
        _check(lib().qsg_set_k_ladder(self.ctx, i, _ptr(k)), self.ctx)

    def tau_overlaps(self, group: int, slots, taus) -> list:
        """Contributions of the configurations now in (group, slots) to the
        Euclidean-time overlaps (qsg_tau_overlaps, one launch): per slot a
        dict of int64 arrays q2, q4 [64][n_taus] and A, B [n_taus][L]; sum
        them over configurations and pass the sums to tau_observables.
        `slots` is a slot index or a range of consecutive slots."""
        torch = self._torch
        slots = range(slots, slots + 1) if isinstance(slots, int) else slots
        if len(slots) == 0 or (len(slots) > 1 and slots.step != 1):
            raise ValueError("slots must be consecutive")
        t = np.ascontiguousarray(np.asarray(taus, dtype=np.uint32))
        L = int(self.descs[group].L)
        n = t.size
        per = n * (128 + 2 * L)
        words = per * len(slots)
        out = torch.zeros(words, dtype=torch.int64, device=self.workspace.device)
        _check(lib().qsg_tau_overlaps(self.ctx, group, slots[0], len(slots), _ptr(t), n,
                                      C.c_void_p(out.data_ptr()), words), self.ctx)
        self.sync()
        res = []
        for a in out.cpu().numpy().reshape(len(slots), per):
            res.append({"q2": a[:64 * n].reshape(64, n), "q4": a[64 * n:128 * n].reshape(64, n),
                        "A": a[128 * n:128 * n + n * L].reshape(n, L),
                        "B": a[128 * n + n * L:].reshape(n, L)})
        return res

    def init_spins(self):
        _check(lib().qsg_init_spins(self.ctx), self.ctx)

    def sweep(self, n: int, flags: int = QSG_PLAIN):
        _check(lib().qsg_sweep(self.ctx, int(n), int(flags)), self.ctx)

    def sweep_status(self, n: int, flags: int = QSG_PLAIN) -> int:
        return int(lib().qsg_sweep(self.ctx, int(n), int(flags)))

    def pt_swap(self):
        _check(lib().qsg_pt_swap(self.ctx), self.ctx)

    def sync(self):
        _check(lib().qsg_sync(self.ctx), self.ctx)

    def set_schedule(self, i: int, sweep_split: int, tau_tile: int | None = None):
        if tau_tile is None:
            _check(lib().qsg_set_schedule(self.ctx, int(i), int(sweep_split)), self.ctx)
        else:
            _check(lib().qsg_set_colour_schedule(self.ctx, int(i), int(sweep_split),
                                                 int(tau_tile)), self.ctx)

    def set_deadline(self, seconds: float):
        _check(lib().qsg_set_deadline(self.ctx, float(seconds)), self.ctx)

    def _measure(self, what, dtype, count):
        out = np.zeros(count, dtype=dtype)
        _check(lib().qsg_measure(self.ctx, what, _ptr(out), out.nbytes), self.ctx)
        return out

    def _split(self, flat, per_group):
        res, off = [], 0
        for i, g in enumerate(self.groups):
            n, shape = per_group(len(g.gammas))
            res.append(flat[off:off + n].reshape(shape))
            off += n
        return res

    def energies(self) -> List[np.ndarray]:
        """[(N, 64, 2) int32 (Bsp, Bt)] recomputed from the current spins."""
        tot = sum(len(g.gammas) * 128 for g in self.groups)
        flat = self._measure(QSG_M_ENERGY, np.int32, tot)
        return self._split(flat, lambda N: (N * 128, (N, 64, 2)))

    def overlaps(self) -> List[np.ndarray]:
        tot = sum(len(g.gammas) * 32 for g in self.groups)
        flat = self._measure(QSG_M_OVERLAP, np.int64, tot)
        return self._split(flat, lambda N: (N * 32, (N, 32)))

    def accepts(self) -> List[np.ndarray]:
        tot = sum(max(len(g.gammas) - 1, 1) for g in self.groups)
        flat = self._measure(QSG_M_ACCEPT, np.uint64, tot)
        return [a[:len(g.gammas) - 1] for a, g in zip(
            self._split(flat, lambda N: (max(N - 1, 1), (max(N - 1, 1),))), self.groups)]

    def walkers(self) -> List[np.ndarray]:
        tot = sum(len(g.gammas) * 64 for g in self.groups)
        flat = self._measure(QSG_M_WALKERS, np.uint8, tot)
        return self._split(flat, lambda N: (N * 64, (N, 64)))

    def swaplog(self) -> List[np.ndarray]:
        cap = self.cfg.swaplog_cap
        tot = sum(cap * max(len(g.gammas) - 1, 1) for g in self.groups)
        flat = self._measure(QSG_M_SWAPLOG, np.uint64, tot)
        return self._split(flat, lambda N: (cap * max(N - 1, 1), (cap, max(N - 1, 1))))

    def swaplog_rows(self) -> List[np.ndarray]:
        """Masks of the PT steps done so far, oldest first (ring order)."""
        p = self.counters()[1]
        cap = self.cfg.swaplog_cap
        n = min(p, cap)
        idx = [(p - n + i) % cap for i in range(n)]
        return [lg[idx].copy() for lg in self.swaplog()]

    def roundtrips(self) -> List[np.ndarray]:
        tot = sum(len(g.gammas) * 64 for g in self.groups)
        flat = self._measure(QSG_M_ROUNDTRIP, ROUNDTRIP_DTYPE, tot)
        return self._split(flat, lambda N: (N * 64, (N, 64)))

    def sums(self) -> List[np.ndarray]:
        tot = sum(len(g.gammas) * SUM_STRIDE for g in self.groups)
        flat = self._measure(QSG_M_SUMS, np.int64, tot)
        return self._split(flat, lambda N: (N * SUM_STRIDE, (N, SUM_STRIDE)))

    def histograms(self) -> List[np.ndarray]:
        tot = sum(len(g.gammas) * HIST_BINS for g in self.groups)
        flat = self._measure(QSG_M_HIST, np.uint32, tot)
        return self._split(flat, lambda N: (N * HIST_BINS, (N, HIST_BINS)))

    def counters(self):
        v = self._measure(QSG_M_COUNTERS, np.uint64, 2)
        return int(v[0]), int(v[1])

    def get_spins(self, i: int) -> np.ndarray:
        g = self.groups[i]
        out = np.zeros(len(g.gammas) * g.L_tau * g.L * g.L, dtype=np.uint64)
        _check(lib().qsg_get_spins(self.ctx, i, _ptr(out), out.size), self.ctx)
        return out

    def set_spins(self, i: int, words: np.ndarray):
        w = np.ascontiguousarray(np.asarray(words, dtype=np.uint64))
        _check(lib().qsg_set_spins(self.ctx, i, _ptr(w), w.size), self.ctx)

    def get_couplings(self, i: int):
        L = self.groups[i].L
        jx = np.zeros(L * L, np.uint64)
        jy = np.zeros(L * L, np.uint64)
        _check(lib().qsg_get_couplings(self.ctx, i, _ptr(jx), _ptr(jy)), self.ctx)
        return jx, jy

    def get_tables(self, i: int):
        N = len(self.groups[i].gammas)
        cap = self.descs[i].swap_table_cap or 4096
        pairs = max(N - 1, 1)
        thr = np.zeros(N * 15, np.uint32)
        eq = np.zeros(pairs, np.uint8)
        ln = np.zeros(pairs, np.uint32)
        sw = np.zeros(pairs * cap, np.uint32)
        _check(lib().qsg_get_tables(self.ctx, i, _ptr(thr), _ptr(eq), _ptr(ln), _ptr(sw)),
               self.ctx)
        return thr.reshape(N, 15), eq[:N - 1], ln[:N - 1], sw.reshape(pairs, cap)[:N - 1]

    def get_state(self) -> np.ndarray:
        n = lib().qsg_state_bytes(self.ctx)
        out = np.zeros(n, np.uint8)
        _check(lib().qsg_get_state(self.ctx, _ptr(out), n), self.ctx)
        return out

    def set_state(self, buf: np.ndarray):
        b = np.ascontiguousarray(buf, dtype=np.uint8)
        _check(lib().qsg_set_state(self.ctx, _ptr(b), b.size), self.ctx)


def philox_device(inputs: np.ndarray) -> np.ndarray:
    """Philox4x32-10 on the GPU for rows (ctr0..3, key0, key1)."""
    import torch
    a = np.ascontiguousarray(np.asarray(inputs, dtype=np.uint32)).reshape(-1, 6)
    d_in = torch.from_numpy(a.view(np.int32).copy()).cuda()
    d_out = torch.zeros((a.shape[0], 4), dtype=torch.int32, device="cuda")
    s = torch.cuda.current_stream()
    _check(lib().qsg_philox(C.c_void_p(d_in.data_ptr()), C.c_void_p(d_out.data_ptr()),
                            a.shape[0], C.c_void_p(s.cuda_stream)))
    torch.cuda.synchronize()
    return d_out.cpu().numpy().view(np.uint32)


def tau_observables(acc: dict, L: int, L_tau: int, n_configs: int) -> dict:
    """Q2(tau), Q4(tau), F(tau) (qsg_tau_observables: App. E normalisation,
    averages over tau1, configurations and the 64 replicas) from summed
    tau_overlaps output of one slot."""
    n = acc["q2"].shape[1]
    sums = np.ascontiguousarray(np.concatenate(
        [np.asarray(acc[k], dtype=np.int64).ravel() for k in ("q2", "q4", "A", "B")]))
    if sums.size != n * (128 + 2 * L):
        raise ValueError("sums do not match L and the number of tau values")
    out = {k: np.zeros(n, dtype=np.float64) for k in ("Q2", "Q4", "F")}
    _check(lib().qsg_tau_observables(_ptr(sums), int(L), int(L_tau), n, int(n_configs),
                                     _ptr(out["Q2"]), _ptr(out["Q4"]), _ptr(out["F"])))
    return out


def philox_probe(out, n_threads: int, blocks: int, key: int, stream) -> None:
    """Enqueue the Philox throughput probe: out is an int32 device tensor of
    n_threads words; stream a torch stream."""
    if out.numel() < n_threads:
        raise ValueError("output tensor too small")
    _check(lib().qsg_philox_probe(n_threads, blocks, key, C.c_void_p(out.data_ptr()),
                                  C.c_void_p(stream.cuda_stream)))


# ------------------------------------------------- transfer matrix (EDQSG)
def tm_desc(L: int, k: float, k_perp: float, jx, jy, parity: int) -> qsg_tm_desc:
    """Descriptor of the slice transfer matrix in one parity sector
    (qsg_tm_apply): couplings jx, jy of +-1 per site j = x1 + L x2."""
    d = qsg_tm_desc()
    d.L, d.parity, d.k, d.k_perp = int(L), int(parity), float(k), float(k_perp)
    jx = np.asarray(jx, dtype=np.int64).ravel()
    jy = np.asarray(jy, dtype=np.int64).ravel()
    if jx.size != L * L or jy.size != L * L:
        raise ValueError("need L*L couplings per direction")
    for j in range(L * L):
        d.jx[j], d.jy[j] = int(jx[j]), int(jy[j])
    return d


def tm_dim(L: int) -> int:
    return int(lib().qsg_tm_dim(L))


def tm_apply(desc: qsg_tm_desc, x, out, stream=None) -> None:
    """out = T x (float64 device tensors of tm_dim(L) entries; x may be out),
    enqueued on `stream` (a torch stream; default the current one)."""
    n = tm_dim(desc.L)
    for t in (x, out):
        if t.dtype != _torch_f64() or not t.is_cuda or t.numel() != n or not t.is_contiguous():
            raise ValueError(f"need contiguous float64 device tensors of {n} entries")
    sp = C.c_void_p(stream.cuda_stream) if stream is not None else _stream_ptr()
    _check(lib().qsg_tm_apply(C.byref(desc), C.c_void_p(x.data_ptr()),
                              C.c_void_p(out.data_ptr()), sp))


def tm_lanczos(desc: qsg_tm_desc, max_iter: int, n_eig: int = 2, tol: float = 1e-10,
               seed: int = 1, want_vector: bool = False, stream=None) -> dict:
    """Largest eigenvalues of the sector (qsg_tm_lanczos): values
    (descending), residual estimates, steps taken and, if asked, the unit
    Ritz vector of the largest (a float64 device tensor)."""
    import torch
    nbytes = int(lib().qsg_tm_lanczos_workspace_bytes(desc.L, max_iter))
    if nbytes == 0:
        raise ValueError("unsupported L or max_iter")
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    vec = torch.empty(tm_dim(desc.L), dtype=torch.float64, device="cuda") if want_vector else None
    eigs = np.zeros(n_eig)
    resid = np.zeros(n_eig)
    iters = np.zeros(1, dtype=np.uint32)
    sp = C.c_void_p(stream.cuda_stream) if stream is not None else _stream_ptr()
    _check(lib().qsg_tm_lanczos(C.byref(desc), max_iter, n_eig, tol, seed,
                                C.c_void_p(ws.data_ptr()), nbytes, _ptr(eigs), _ptr(resid),
                                _ptr(iters), _dp(vec), sp))
    return {"values": eigs, "resid": resid, "iters": int(iters[0]), "vector": vec}


def tm_correlations(L: int, vec, stream=None) -> dict:
    """Ground-state correlations Q2, Q4, F of a sector vector (a float64
    device tensor of tm_dim(L) entries; qsg_tm_correlations) and the
    second-moment correlation length sqrt(Q2/F - 1) / (2 sin(pi/L))."""
    import math
    import torch
    n = tm_dim(L)
    if vec.dtype != torch.float64 or not vec.is_cuda or vec.numel() != n or not vec.is_contiguous():
        raise ValueError(f"need a contiguous float64 device tensor of {n} entries")
    nbytes = int(lib().qsg_tm_correlations_workspace_bytes(L))
    ws = torch.empty(nbytes, dtype=torch.uint8, device=vec.device)
    out = np.zeros(3)
    sp = C.c_void_p(stream.cuda_stream) if stream is not None else _stream_ptr()
    _check(lib().qsg_tm_correlations(L, C.c_void_p(vec.data_ptr()), C.c_void_p(ws.data_ptr()),
                                     nbytes, _ptr(out), sp))
    q2, q4, f = (float(v) for v in out)
    xi = math.sqrt(q2 / f - 1.0) / (2.0 * math.sin(math.pi / L)) if f > 0 and q2 > f else float("nan")
    return {"Q2": q2, "Q4": q4, "F": f, "xi2": xi}


def tm_correlations_lt(L: int, v_even, v_odd, lambda_even: float, lambda_odd: float,
                       l_taus, stream=None) -> list:
    """Finite-L_tau estimates of Q2, Q4, F from the leading even and odd
    states (float64 device tensors of tm_dim(L) entries and their
    eigenvalues) for each length in l_taus (0: L_tau -> infinity);
    qsg_tm_correlations_lt.  One dict per length, as tm_correlations."""
    import math
    import torch
    n = tm_dim(L)
    for v in (v_even, v_odd):
        if v.dtype != torch.float64 or not v.is_cuda or v.numel() != n or not v.is_contiguous():
            raise ValueError(f"need contiguous float64 device tensors of {n} entries")
    lt = np.ascontiguousarray(np.asarray(l_taus, dtype=np.uint32).reshape(-1))
    nbytes = int(lib().qsg_tm_correlations_lt_workspace_bytes(L, len(lt)))
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=v_even.device)
    out = np.zeros(3 * max(len(lt), 1))
    sp = C.c_void_p(stream.cuda_stream) if stream is not None else _stream_ptr()
    _check(lib().qsg_tm_correlations_lt(L, C.c_void_p(v_even.data_ptr()),
                                        C.c_void_p(v_odd.data_ptr()), float(lambda_even),
                                        float(lambda_odd), _ptr(lt), len(lt),
                                        C.c_void_p(ws.data_ptr()), nbytes, _ptr(out), sp))
    res = []
    for i in range(len(lt)):
        q2, q4, f = (float(v) for v in out[3 * i:3 * i + 3])
        xi = (math.sqrt(q2 / f - 1.0) / (2.0 * math.sin(math.pi / L))
              if f > 0 and q2 > f else float("nan"))
        res.append({"L_tau": int(lt[i]), "Q2": q2, "Q4": q4, "F": f, "xi2": xi})
    return res


def _torch_f64():
    import torch
    return torch.float64


# ------------------------------------------------------------- ladder MLP
def _dp(t) -> C.c_void_p:
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _stream_ptr():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def qsg_mlp_forward(params, params_bf16, x, out, ws):
    _check(lib().qsg_mlp_forward(_dp(params), _dp(params_bf16), _dp(x), x.shape[0], _dp(out),
                                 _dp(ws), _stream_ptr()))


def qsg_mlp_forward_noalloc(params, params_bf16, x, out):
    _check(lib().qsg_mlp_forward_noalloc(_dp(params), _dp(params_bf16), _dp(x), x.shape[0],
                                         _dp(out), _stream_ptr()))


def qsg_mlp_backward(params, params_bf16, x, ws, dout, grads, scratch):
    _check(lib().qsg_mlp_backward(_dp(params), _dp(params_bf16), _dp(x), _dp(ws), _dp(dout),
                                  x.shape[0], _dp(grads), _dp(scratch), _stream_ptr()))


def qsg_mlp_loss(z, t, logL, dz, loss):
    _check(lib().qsg_mlp_loss(_dp(z), _dp(t), _dp(logL), z.shape[0], _dp(dz), _dp(loss),
                              _stream_ptr()))


def qsg_mlp_adam(params, params_bf16, grads, m, v, step, lr):
    _check(lib().qsg_mlp_adam(_dp(params), _dp(params_bf16), _dp(grads), _dp(m), _dp(v),
                              int(step), float(lr), _stream_ptr()))


def qsg_mlp_to_bf16(params, params_bf16):
    _check(lib().qsg_mlp_to_bf16(_dp(params), _dp(params_bf16), _stream_ptr()))


def qsg_mlp_decode(z, gmin, gmax, ladder, acc_pred=None):
    _check(lib().qsg_mlp_decode(_dp(z), _dp(gmin), _dp(gmax), z.shape[0], _dp(ladder),
                                _dp(acc_pred), _stream_ptr()))
