"""GPU checks of the ladder MLP kernels against the float64 oracle.

FP32 path (no BF16 copy): forward and gradients within 1e-5 relative; BF16
path: within 1e-2 relative (operand rounding to bfloat16 can differ where the
two sides' FP32/FP64 values straddle a rounding boundary).  Plus: decode,
Adam, a training run whose loss falls, and the learned ladder's gain over the
geometric ladder on a small ensemble.
"""
import math

import numpy as np
import pytest

import qsg_workloads as W
from oracle import mlp as omlp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2402_03920_amd import ladder, qsg  # noqa: E402


def _data(B=37, seed=2):
    rng = np.random.Generator(np.random.PCG64(seed))
    X = rng.normal(size=(B, 6)).astype(np.float32)
    t = rng.random((B, 31)) + 0.02
    t = (t / t.sum(axis=1, keepdims=True)).astype(np.float32)
    logL = rng.normal(size=B).astype(np.float32)
    return X, t, logL


def _rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-30)


@pytest.mark.parametrize("bf16,tol", [(False, 1e-5), (True, 1e-2)])
def test_forward_loss_backward_match_oracle(bf16, tol):
    p = ladder.init_params(1).astype(np.float64)
    p[-32:] += 0.3  # non-trivial output bias
    X, t, logL = _data()
    # the oracle sees exactly the FP32 parameters the GPU holds
    p32 = p.astype(np.float32).astype(np.float64)
    net = ladder.LadderMLP(bf16=bf16, params=p32)
    x = torch.tensor(X, device="cuda")
    out, ws = net.forward(x)
    cache = omlp.forward(p32, X.astype(np.float64), bf16=bf16)
    assert _rel(out.cpu().numpy(), cache["out"]) < tol
    dz = torch.empty_like(out)
    loss = torch.empty(X.shape[0], device="cuda")
    qsg.qsg_mlp_loss(out, torch.tensor(t, device="cuda"), torch.tensor(logL, device="cuda"), dz, loss)
    oloss, odz = omlp.loss_and_grad(cache["out"], t.astype(np.float64), logL.astype(np.float64))
    assert abs(float(loss.mean()) - oloss) / abs(oloss) < tol
    assert _rel(dz.cpu().numpy(), odz) < tol
    # backward from the same output gradient on both sides
    dz_in = torch.tensor(odz.astype(np.float32), device="cuda")
    grads = torch.zeros(net.n_params, device="cuda")
    scratch = torch.empty(2 * X.shape[0] * 128, device="cuda")
    qsg.qsg_mlp_backward(net.params, net.bf16, x, ws, dz_in, grads, scratch)
    og = omlp.backward(p32, cache, odz.astype(np.float32).astype(np.float64), bf16=bf16)
    g = grads.cpu().numpy()
    off = 0
    for k, n in omlp.SIZES:  # every layer separately, weights and biases
        for size in (k * n, n):
            assert _rel(g[off:off + size], og[off:off + size]) < tol, (k, n, size)
            off += size


def test_adam_matches_oracle():
    p = ladder.init_params(3).astype(np.float64)
    p32 = p.astype(np.float32).astype(np.float64)
    net = ladder.LadderMLP(bf16=True, params=p32)
    rng = np.random.Generator(np.random.PCG64(4))
    m = np.zeros_like(p32)
    v = np.zeros_like(p32)
    cur = p32.copy()
    for step in (1, 2, 3):
        g = rng.normal(size=p.size).astype(np.float32)
        net.grads.copy_(torch.tensor(g, device="cuda"))
        net.step = step - 1
        qsg.qsg_mlp_adam(net.params, net.bf16, net.grads, net.m, net.v, step, 1e-3)
        cur, m, v = omlp.adam(cur, g.astype(np.float64), m, v, step, 1e-3)
    assert _rel(net.params.cpu().numpy(), cur) < 1e-5
    bf = net.bf16.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    assert np.array_equal(bf.view(np.float32), omlp.to_bf16(net.params.cpu().numpy()).astype(np.float32))


def test_decode_matches_oracle_and_zero_logits_are_geometric():
    rng = np.random.Generator(np.random.PCG64(5))
    z = rng.normal(scale=2.0, size=(9, 32)).astype(np.float32)
    z[0] = 0.0
    gmin = np.full(9, 2.0)
    gmax = np.full(9, 4.0)
    zt = torch.tensor(z, device="cuda")
    lad = torch.empty((9, 32), dtype=torch.float64, device="cuda")
    acc = torch.empty(9, device="cuda")
    qsg.qsg_mlp_decode(zt, torch.tensor(gmin, device="cuda"), torch.tensor(gmax, device="cuda"),
                       lad, acc)
    got = lad.cpu().numpy()
    want = omlp.decode(z.astype(np.float64), gmin, gmax)
    assert np.max(np.abs(got - want) / want) < 1e-12
    assert np.allclose(got[0], W.geometric_ladder(2.0, 4.0, 32), rtol=1e-13)
    assert np.all(np.diff(got, axis=1) >= 0) and np.all(got[:, 0] == 2.0) and np.all(got[:, -1] == 4.0)
    assert np.allclose(acc.cpu().numpy(), omlp.predicted_acceptance(z), atol=1e-6)


def test_training_reduces_the_loss():
    X, t, logL = _data(B=64, seed=7)
    net = ladder.LadderMLP(seed=0, bf16=True)
    hist = net.fit(X, t, logL, steps=300, lr=2e-3, log_every=50)
    assert hist[-1] < 0.5 * hist[0]


def test_uniform_acceptance_targets_are_the_geometric_ladder():
    lad = W.geometric_ladder(2.0, 4.0, 24)
    inc, logL = ladder.targets_from_acceptance(lad, np.full(23, 0.6))
    assert np.allclose(inc, 1.0 / 31, atol=1e-6)
    assert abs(logL - math.log(23 * 0.4)) < 1e-9
