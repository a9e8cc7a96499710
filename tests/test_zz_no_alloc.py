"""The allocation-free MLP forward (qsg_mlp_forward_noalloc) against the
forward with a caller workspace (qsg_mlp_forward), through the C ABI: equal
bit for bit on two calls in a row, the second with a smaller batch (the
fixed array keeps the first call's contents), both weight forms; batches
over the limit are refused before any launch."""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2402_03920_amd import ladder, qsg  # noqa: E402


def _forward_ws(net, x):
    B = x.shape[0]
    ws = torch.empty(int(qsg.lib().qsg_mlp_workspace_floats(B)), dtype=torch.float32,
                     device="cuda")
    out = torch.empty((B, 32), dtype=torch.float32, device="cuda")
    qsg.qsg_mlp_forward(net.params, net.bf16, x, out, ws)
    return out


def _forward_noalloc(net, x):
    out = torch.full((x.shape[0], 32), float("nan"), dtype=torch.float32, device="cuda")
    qsg.qsg_mlp_forward_noalloc(net.params, net.bf16, x, out)
    return out


@pytest.mark.parametrize("bf16", [True, False])
def test_noalloc_forward_equals_workspace_forward(bf16):
    net = ladder.LadderMLP(seed=3, bf16=bf16)
    rng = np.random.Generator(np.random.PCG64(11))
    for B in (1024, 37):  # the limit, then a smaller batch
        x = torch.tensor(rng.normal(size=(B, 6)).astype(np.float32), device="cuda")
        want = _forward_ws(net, x)
        got = _forward_noalloc(net, x)
        torch.cuda.synchronize()
        assert torch.equal(got, want), B
    # batches the fixed array cannot hold are refused, nothing launched
    x = torch.zeros((1025, 6), dtype=torch.float32, device="cuda")
    out = torch.zeros((1025, 32), dtype=torch.float32, device="cuda")
    with pytest.raises(qsg.QSGError) as e:
        qsg.qsg_mlp_forward_noalloc(net.params, net.bf16, x, out)
    assert e.value.code == qsg.QSG_E_INVALID
    assert torch.count_nonzero(out).item() == 0
