"""CPU checks of the C ABI: the library loads, exports every declared
symbol, validates its arguments, and its binary128 tables equal the
oracle's mpmath tables entry for entry (no GPU needed for any of these)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import qsg_workloads as W
from oracle import tables
from paper_2402_03920_amd import qsg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"\b(qsg_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = qsg.lib()
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n


def _desc(**kw):
    d = dict(L=8, L_tau=32, beta=4.0, n_gamma=16, group_id=0, mc_seed=42, j_seeds=[1] * 64)
    d.update(kw)
    return qsg.make_desc(**d)


def _ws_bytes(desc, pt_every=10, cap=128):
    arr = (qsg.qsg_group_desc * 1)(desc)
    cfg = qsg.qsg_run_config(pt_every, cap, 0, 0)
    return qsg.lib().qsg_workspace_bytes(arr, 1, C.byref(cfg))


def test_workspace_validation():
    assert _ws_bytes(_desc()) > 16 * 32 * 64 * 8
    for bad in (dict(L=7), dict(L=0), dict(L_tau=3), dict(n_gamma=0), dict(n_gamma=65),
                dict(beta=-1.0), dict(beta=float("nan"))):
        assert _ws_bytes(_desc(**bad)) == 0, bad
    assert _ws_bytes(_desc(), cap=0) == 0


def test_create_rejects_bad_workspace_without_touching_the_device():
    arr = (qsg.qsg_group_desc * 1)(_desc())
    cfg = qsg.qsg_run_config(10, 16, 0, 0)
    out = C.c_void_p()
    rc = qsg.lib().qsg_create(arr, 1, C.byref(cfg), None, 0, None, C.byref(out))
    assert rc == qsg.QSG_E_INVALID and not out.value
    assert b"workspace" in qsg.lib().qsg_last_error(None)
    rc = qsg.lib().qsg_create(arr, 1, C.byref(cfg), C.c_void_p(4096), 16, None, C.byref(out))
    assert rc == qsg.QSG_E_BUFFER


def test_host_tables_reject_bad_ladders():
    with pytest.raises(qsg.QSGError) as e:
        qsg.qsg_build_tables(4.0, 32, [2.0, 1.0])
    assert e.value.code == qsg.QSG_E_INVALID
    with pytest.raises(qsg.QSGError) as e:
        qsg.qsg_build_tables(4.0, 32, [1.0, -1.0])
    assert e.value.code == qsg.QSG_E_INVALID
    # a tiny gap needs a long exchange table
    with pytest.raises(qsg.QSGError) as e:
        qsg.qsg_build_tables(128.0, 2048, [3.0, 3.0 + 1e-7], cap=64)
    assert e.value.code == qsg.QSG_E_UNSUPPORTED


def _ladders():
    out = []
    for g in W.plain_small().groups:
        out.append((g.beta, g.L_tau, g.gammas))
    out.append((8.0, 128, W.geometric_ladder(2.0, 4.0, 32)))             # c2
    for Lt, ng in ((64, 24), (128, 37), (256, 48)):                        # c3 shapes
        out.append((Lt / 16.0, Lt, W.geometric_ladder(2.0, 4.0, ng)))
    out.append((128.0, 2048, W.geometric_ladder(2.8, 3.6, 48)))          # c4
    out.append((16.0, 256, W.geometric_ladder(2.0, 4.0, 32)))            # c5
    out.append((1.0, 4, np.array([0.5, 0.5, 1.0, 60.0])))                 # equal pair, kp ~ 0
    out.append((1.0, 4, np.array([1e-6, 0.3])))                           # frozen limit
    return out


@pytest.mark.parametrize("case", range(len(_ladders())))
def test_binary128_tables_equal_oracle_mpmath(case):
    beta, Lt, lad = _ladders()[case]
    cap = 8192
    thr, eq, ln, sw = qsg.qsg_build_tables(beta, Lt, lad, cap=cap)
    othr = tables.metropolis_thresholds(beta, Lt, lad).reshape(len(lad), 15)
    assert np.array_equal(thr, othr)
    oeq, oln, otabs = tables.swap_tables(beta, Lt, lad)
    assert np.array_equal(eq, oeq)
    assert np.array_equal(ln, oln)
    for g, t in enumerate(otabs):
        assert np.array_equal(sw[g, :len(t)], t)
        assert np.all(sw[g, len(t):] == 0)


def test_ladder_kind_is_validated():
    assert _ws_bytes(_desc(ladder="k")) > 0
    d = _desc()
    d.ladder_kind = 2
    assert _ws_bytes(d) == 0


def test_host_k_tables_reject_bad_ladders():
    for bad in ([0.2, 0.3], [0.3, -0.1], [0.3, float("nan")]):
        with pytest.raises(qsg.QSGError) as e:
            qsg.qsg_build_tables_k(bad)
        assert e.value.code == qsg.QSG_E_INVALID, bad
    with pytest.raises(qsg.QSGError) as e:
        qsg.qsg_build_tables_k([0.3, 0.3 - 1e-9], cap=64)
    assert e.value.code == qsg.QSG_E_UNSUPPORTED


def _k_ladders():
    return [W.coupling_ladder(1).groups[0].gammas,            # 32 k in [0.25, 0.33]
            W.linear_k_ladder(0.5, 0.2, 3),
            np.array([0.4, 0.4, 0.3, 0.05]),                       # equal pair
            np.array([2.5, 1e-3])]                                 # saturated and tiny k


@pytest.mark.parametrize("case", range(len(_k_ladders())))
def test_binary128_k_tables_equal_oracle_mpmath(case):
    lad = _k_ladders()[case]
    cap = 8192
    thr, eq, ln, sw = qsg.qsg_build_tables_k(lad, cap=cap)
    othr = tables.metropolis_thresholds_k(lad).reshape(len(lad), 15)
    assert np.array_equal(thr, othr)
    oeq, oln, otabs = tables.swap_tables_k(lad)
    assert np.array_equal(eq, oeq)
    assert np.array_equal(ln, oln)
    for g, t in enumerate(otabs):
        assert np.array_equal(sw[g, :len(t)], t)
        assert np.all(sw[g, len(t):] == 0)


def test_tau_boundary_is_validated():
    assert _ws_bytes(_desc(antiperiodic=True)) > 0
    d = _desc()
    d.tau_boundary = 2
    assert _ws_bytes(d) == 0
    d = _desc()
    d.reserved = 1
    assert _ws_bytes(d) == 0


def test_transfer_matrix_sizes_and_validation_without_the_device():
    """qsg_tm_dim / workspace sizes, and descriptor checks that fail before
    any launch (L out of range, parity, couplings, null vectors)."""
    from paper_2402_03920_amd import qsg
    lib = qsg.lib()
    assert [lib.qsg_tm_dim(L) for L in range(1, 8)] == [0, 8, 256, 1 << 15, 1 << 24, 0, 0]
    assert lib.qsg_tm_lanczos_workspace_bytes(4, 0) == 0
    assert lib.qsg_tm_lanczos_workspace_bytes(6, 10) == 0
    n = lib.qsg_tm_lanczos_workspace_bytes(3, 10)
    assert n >= 12 * 256 * 8 and n % 8 == 0
    j = [1] * 9
    dummy = C.c_void_p(1)  # never dereferenced: every case fails validation first
    cases = [(qsg.tm_desc(3, 0.3, 0.3, j, j, 1), None, qsg.QSG_E_INVALID),
             (qsg.tm_desc(3, 0.3, 0.3, j, j, 0), dummy, qsg.QSG_E_INVALID),
             (qsg.tm_desc(3, 0.3, float("nan"), j, j, 1), dummy, qsg.QSG_E_INVALID),
             (qsg.tm_desc(3, 0.3, 0.3, [1] * 8 + [0], j, 1), dummy, qsg.QSG_E_INVALID)]
    big = qsg.tm_desc(5, 0.3, 0.3, [1] * 25, [1] * 25, 1)
    big.L = 6
    cases.append((big, dummy, qsg.QSG_E_UNSUPPORTED))
    small = qsg.tm_desc(2, 0.3, 0.3, [1] * 4, [1] * 4, 1)
    small.L = 1
    cases.append((small, dummy, qsg.QSG_E_INVALID))
    for d, ptr, want in cases:
        rc = lib.qsg_tm_apply(C.byref(d), ptr, ptr, None)
        assert rc == want, (d.L, d.parity, rc)
        assert lib.qsg_last_error(None)
    d = qsg.tm_desc(3, 0.3, 0.3, j, j, 1)
    out = np.zeros(2)
    it = np.zeros(1, dtype=np.uint32)
    for max_iter, n_eig, ws in ((0, 1, 1 << 20), (10, 0, 1 << 20), (10, 11, 1 << 20), (10, 2, 8)):
        rc = lib.qsg_tm_lanczos(C.byref(d), max_iter, n_eig, 1e-10, 1, dummy, ws, out.ctypes.data,
                                out.ctypes.data, it.ctypes.data, None, None)
        assert rc in (qsg.QSG_E_INVALID, qsg.QSG_E_BUFFER), (max_iter, n_eig, ws, rc)


def test_correlations_sizes_and_validation_without_the_device():
    from paper_2402_03920_amd import qsg
    lib = qsg.lib()
    assert lib.qsg_tm_correlations_workspace_bytes(1) == 0
    assert lib.qsg_tm_correlations_workspace_bytes(6) == 0
    assert lib.qsg_tm_correlations_workspace_bytes(5) >= (1 << 24) * 8 + 12950 * 28
    out = np.zeros(3)
    dummy = C.c_void_p(1)  # never dereferenced: every case fails validation first
    big = lib.qsg_tm_correlations_workspace_bytes(3)
    for L, vec, ws, nbytes, want in ((1, dummy, dummy, big, qsg.QSG_E_INVALID),
                                     (6, dummy, dummy, big, qsg.QSG_E_UNSUPPORTED),
                                     (3, None, dummy, big, qsg.QSG_E_INVALID),
                                     (3, dummy, None, big, qsg.QSG_E_INVALID),
                                     (3, dummy, dummy, 16, qsg.QSG_E_BUFFER)):
        rc = lib.qsg_tm_correlations(L, vec, ws, nbytes, out.ctypes.data, None)
        assert rc == want, (L, rc)


def test_finite_length_correlations_validation_without_the_device():
    from paper_2402_03920_amd import qsg
    lib = qsg.lib()
    assert lib.qsg_tm_correlations_lt_workspace_bytes(3, 0) == 0
    assert lib.qsg_tm_correlations_lt_workspace_bytes(3, 4097) == 0
    assert lib.qsg_tm_correlations_lt_workspace_bytes(6, 1) == 0
    one = lib.qsg_tm_correlations_lt_workspace_bytes(3, 1)
    assert one >= lib.qsg_tm_correlations_workspace_bytes(3) + 8 * lib.qsg_tm_dim(3)
    assert lib.qsg_tm_correlations_lt_workspace_bytes(3, 100) > one
    lt = np.array([0, 8, 64], dtype=np.uint32)
    out = np.zeros(9)
    dummy = C.c_void_p(1)  # never dereferenced: every case fails validation first
    big = lib.qsg_tm_correlations_lt_workspace_bytes(3, 3)
    cases = ((1, 1.0, 0.5, 3, big, qsg.QSG_E_INVALID),
             (6, 1.0, 0.5, 3, big, qsg.QSG_E_UNSUPPORTED),
             (3, 1.0, 0.5, 0, big, qsg.QSG_E_INVALID),
             (3, 0.0, 0.5, 3, big, qsg.QSG_E_INVALID),
             (3, 1.0, -0.5, 3, big, qsg.QSG_E_INVALID),
             (3, float("inf"), 0.5, 3, big, qsg.QSG_E_INVALID),
             (3, float("nan"), 0.5, 3, big, qsg.QSG_E_INVALID),
             (3, 1.0, 0.5, 3, 16, qsg.QSG_E_BUFFER))
    for L, le, lo, n, nbytes, want in cases:
        rc = lib.qsg_tm_correlations_lt(L, dummy, dummy, le, lo, lt.ctypes.data, n, dummy, nbytes,
                                        out.ctypes.data, None)
        assert rc == want, (L, le, lo, n, rc)
    rc = lib.qsg_tm_correlations_lt(3, None, dummy, 1.0, 0.5, lt.ctypes.data, 3, dummy, big,
                                    out.ctypes.data, None)
    assert rc == qsg.QSG_E_INVALID


def test_binding_fails_loudly_without_the_library(monkeypatch, tmp_path):
    """No fallback: with the shared library absent every entry point raises
    instead of computing anything on the host."""
    from paper_2402_03920_amd import qsg
    monkeypatch.setattr(qsg, "_lib", None)
    monkeypatch.setattr(qsg, "LIB_PATH", str(tmp_path / "libqsg.so"))
    with pytest.raises(ImportError, match="missing"):
        qsg.lib()
    with pytest.raises(ImportError):
        qsg.tm_dim(3)


def test_slot_size_limit_is_enforced_without_touching_the_device():
    """A slot of more than 2^29 words is refused (32-bit byte offsets and
    32-bit bond sums): qsg_workspace_bytes gives 0 and qsg_create returns
    QSG_E_UNSUPPORTED with no context; exactly 2^29 words is accepted."""
    at_limit = _desc(L=256, L_tau=8192, n_gamma=1)
    assert _ws_bytes(at_limit) > (1 << 29) * 8
    over = _desc(L=256, L_tau=16384, n_gamma=1)
    assert _ws_bytes(over) == 0
    arr = (qsg.qsg_group_desc * 1)(over)
    cfg = qsg.qsg_run_config(10, 16, 0, 0)
    out = C.c_void_p()
    rc = qsg.lib().qsg_create(arr, 1, C.byref(cfg), C.c_void_p(4096), 1 << 40, None,
                              C.byref(out))
    assert rc == qsg.QSG_E_UNSUPPORTED and not out.value
    assert b"2^29" in qsg.lib().qsg_last_error(None)
    # groups that together need 2^31 or more blocks in one pass
    many = (qsg.qsg_group_desc * 64)(*([_desc(L=256, L_tau=8192, n_gamma=64)] * 64))
    assert qsg.lib().qsg_workspace_bytes(many, 64, C.byref(cfg)) == 0
    rc = qsg.lib().qsg_create(many, 64, C.byref(cfg), C.c_void_p(4096), 1 << 62, None,
                              C.byref(out))
    assert rc == qsg.QSG_E_UNSUPPORTED and not out.value


def test_tau_observables_follow_the_normalisation_without_the_device():
    """qsg_tau_observables (host code of the library): App. E's averages over
    tau1, configurations and replicas of summed integer overlaps, against
    the oracle's observables on random sums, and its argument checks."""
    import numpy as np
    from oracle import overlaps
    from paper_2402_03920_amd import qsg
    rng = np.random.default_rng(12)
    for L, L_tau, n, confs in ((4, 8, 3, 1), (6, 10, 5, 7), (32, 64, 2, 2)):
        acc = {"q2": rng.integers(0, 10 ** 9, (64, n)), "q4": rng.integers(0, 10 ** 15, (64, n)),
               "A": rng.integers(-10 ** 6, 10 ** 6, (n, L)),
               "B": rng.integers(-10 ** 6, 10 ** 6, (n, L))}
        got = qsg.tau_observables(acc, L, L_tau, confs)
        want = overlaps.observables(acc, L, L_tau, confs)
        for key in ("Q2", "Q4"):
            assert np.allclose(got[key], want[key], rtol=1e-13, atol=0), key
        assert np.allclose(got["F"], want["F"], rtol=1e-12, atol=1e-9)
    f = qsg.lib().qsg_tau_observables
    buf = np.zeros(2 * 128 + 4 * 4, dtype=np.int64)
    out = np.zeros(2)
    p = qsg._ptr
    assert f(p(buf), 4, 8, 2, 0, p(out), p(out), p(out)) == qsg.QSG_E_INVALID
    assert f(p(buf), 0, 8, 2, 1, p(out), p(out), p(out)) == qsg.QSG_E_INVALID
    assert f(None, 4, 8, 2, 1, p(out), p(out), p(out)) == qsg.QSG_E_INVALID
    assert f(p(buf), 4, 8, 2, 1, p(out), p(out), p(out)) == qsg.QSG_OK
