"""The allocation-free gradient call (lbml_loss_grad_static) against lbml_loss_grad.

The library's own work array replaces the caller's work buffer; both calls run
the same kernels on the same inputs, so the gradient and the loss agree bit for
bit.  Two calls in a row, the second with fewer samples than the first (the
array keeps the first call's contents), and the size limit.
"""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_0707_1299_amd import lbm, mobility  # noqa: E402


def _inputs(n, seed):
    g = np.random.default_rng(seed)
    x = torch.tensor(g.uniform(-1, 1, size=(n, 4)).astype(np.float32), device="cuda")
    y = torch.tensor(g.normal(scale=0.3, size=n).astype(np.float32), device="cuda")
    return x, y


def test_static_work_matches_caller_work_on_two_calls():
    master = torch.tensor(mobility.init_master(3), device="cuda")
    w16 = torch.zeros(lbm.LBML_NPARAM, dtype=torch.int16, device="cuda")
    lbm.lbml_round_bf16(master, w16)
    for n, seed in ((3000, 1), (517, 2)):
        x, y = _inputs(n, seed)
        g_ref = torch.zeros(lbm.LBML_NPARAM, dtype=torch.float32, device="cuda")
        l_ref = torch.zeros(1, dtype=torch.float32, device="cuda")
        work = torch.empty(lbm.lbml_work_floats(n), dtype=torch.float32, device="cuda")
        lbm.lbml_loss_grad(w16, x, y, g_ref, l_ref, work)
        g = torch.full((lbm.LBML_NPARAM,), float("nan"), dtype=torch.float32, device="cuda")
        loss = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
        lbm.lbml_loss_grad_static(w16, x, y, g, loss)
        torch.cuda.synchronize()
        print("n=%d: loss %.6e, max |grad| %.3e" % (n, loss.item(), g.abs().max().item()))
        assert torch.equal(g, g_ref)
        assert torch.equal(loss, l_ref)


def test_static_work_size_limit():
    w16 = torch.zeros(lbm.LBML_NPARAM, dtype=torch.int16, device="cuda")
    n = lbm.LBML_STATIC_MAX_N + 1
    x, y = _inputs(n, 3)
    g = torch.zeros(lbm.LBML_NPARAM, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    with pytest.raises(lbm.LBError) as e:
        lbm.lbml_loss_grad_static(w16, x, y, g, loss)
    assert e.value.status == lbm.LB_ERR_SIZE
    # the largest size is accepted
    x, y = _inputs(lbm.LBML_STATIC_MAX_N, 4)
    lbm.lbml_loss_grad_static(w16, x, y, g, loss)
    torch.cuda.synchronize()
    assert np.isfinite(loss.item())
    lib = ctypes.CDLL(lbm.LIB_PATH)
    assert hasattr(lib, "lbml_loss_grad_static")
