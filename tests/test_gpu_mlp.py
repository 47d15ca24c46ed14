"""GPU parity of the mobility-correction network kernels against the FP64
oracle (oracle/mlp.py), and of the colloid update that evaluates it inline.

bf16 rounding is an integer decision taken by both sides from the same
float32 master values: bit-exact.  Forward, gradient and Adam run in FP32 on
the GPU and FP64 in the oracle: relative bounds below come from FP32
accumulation over at most 64-term dot products and n-term sample sums.
"""
import numpy as np
import pytest

import oracle
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_0707_1299_amd import lbm, mobility  # noqa: E402


def _bits_to_f32(w16):
    return (w16.cpu().numpy().astype(np.uint16).astype(np.uint32) << 16).view(np.float32)


def _setup(n=300, seed=0):
    g = np.random.default_rng(seed)
    master = (omlp.init_params(seed) + g.normal(scale=0.05, size=omlp.NPARAM)).astype(np.float32)
    X = g.uniform(-1, 1, size=(n, 4)).astype(np.float32)
    y = (0.3 * np.sin(2 * X[:, 0]) * np.cos(X[:, 1]) + 0.1 * X[:, 3]).astype(np.float32)
    return master, X, y


def test_round_bf16_bit_exact():
    master, _, _ = _setup()
    master[:5] = [1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -(1.0 + 2 ** -8 + 2 ** -20), 3.0e-3, 0.0]
    w16 = torch.zeros(lbm.LBML_NPARAM, dtype=torch.int16, device="cuda")
    lbm.lbml_round_bf16(torch.tensor(master, device="cuda"), w16)
    assert np.array_equal(_bits_to_f32(w16).astype(np.float64), omlp.bf16_round(master))


def test_forward_matches_oracle():
    master, X, _ = _setup()
    w16 = torch.zeros(lbm.LBML_NPARAM, dtype=torch.int16, device="cuda")
    lbm.lbml_round_bf16(torch.tensor(master, device="cuda"), w16)
    y = torch.empty(len(X), dtype=torch.float32, device="cuda")
    lbm.lbml_forward(w16, torch.tensor(X, device="cuda"), y)
    ref, _ = omlp.forward(master, X)
    assert np.abs(y.cpu().numpy() - ref).max() <= 2e-6 * max(1.0, np.abs(ref).max())


def test_loss_grad_matches_oracle_and_is_deterministic():
    master, X, y = _setup(n=517)
    dm = torch.tensor(master, device="cuda")
    w16 = torch.zeros(lbm.LBML_NPARAM, dtype=torch.int16, device="cuda")
    lbm.lbml_round_bf16(dm, w16)
    n = len(X)
    grad = torch.zeros(lbm.LBML_NPARAM, dtype=torch.float32, device="cuda")
    grad2 = torch.zeros_like(grad)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    work = torch.empty(lbm.lbml_work_floats(n), dtype=torch.float32, device="cuda")
    xd, yd = torch.tensor(X, device="cuda"), torch.tensor(y, device="cuda")
    lbm.lbml_loss_grad(w16, xd, yd, grad, loss, work)
    lbm.lbml_loss_grad(w16, xd, yd, grad2, loss, work)
    assert torch.equal(grad, grad2)
    l_ref, g_ref = omlp.loss_and_grad(master, X, y, round_bf16=True)
    assert abs(loss.item() - l_ref) <= 1e-5 * l_ref
    g = grad.cpu().numpy().astype(np.float64)
    assert np.abs(g - g_ref).max() <= 1e-4 * np.abs(g_ref).max()


def test_adam_step_matches_oracle():
    master, X, y = _setup(n=64)
    g = np.random.default_rng(5).normal(size=omlp.NPARAM).astype(np.float32)
    m0 = np.random.default_rng(6).normal(scale=0.1, size=omlp.NPARAM).astype(np.float32)
    v0 = np.abs(np.random.default_rng(7).normal(scale=0.1, size=omlp.NPARAM)).astype(np.float32)
    dm, dmm, dv = (torch.tensor(a, device="cuda") for a in (master, m0, v0))
    w16 = torch.zeros(lbm.LBML_NPARAM, dtype=torch.int16, device="cuda")
    lbm.lbml_adam_step(dm, dmm, dv, torch.tensor(g, device="cuda"), w16, 7, lr=1e-3)
    ref, mr, vr = omlp.adam_step(master.astype(np.float64), m0.astype(np.float64), v0.astype(np.float64),
                                 g.astype(np.float64), 7, lr=1e-3)
    assert np.abs(dm.cpu().numpy() - ref).max() <= 1e-6
    assert np.abs(dmm.cpu().numpy() - mr).max() <= 1e-6 * np.abs(mr).max()
    assert np.abs(dv.cpu().numpy() - vr).max() <= 1e-6 * np.abs(vr).max()
    assert np.array_equal(_bits_to_f32(w16).astype(np.float64), omlp.bf16_round(dm.cpu().numpy()))


def test_training_reduces_loss_on_device():
    g = np.random.default_rng(8)
    offs = g.uniform(0, 1, size=(400, 3))
    taus = g.uniform(0.6, 1.5, size=400)
    mu = 0.7 + 0.01 * np.cos(2 * np.pi * offs[:, 0]) * np.cos(2 * np.pi * offs[:, 1]) + 0.02 * (taus - 1)
    tr = mobility.train(offs, taus, mu, iters=1500, lr=3e-3)
    assert tr.losses[-1][1] < 0.05 * tr.losses[0][1]
    pred = mobility.predict(tr, offs, taus)
    assert np.sqrt(np.mean((pred - mu) ** 2)) < 0.2 * np.sqrt(np.mean((mu - mu.mean()) ** 2))


def test_colloid_update_with_inline_mlp_matches_oracle():
    """Advected colloids whose 1/a_L comes from the network, FP64 lattice, against the
    oracle evaluating the same bf16 network in FP64."""
    shape = (20, 20, 24)
    g = np.random.default_rng(9)
    pos = g.uniform(0, 1, (6, 3)) * np.array([24, 20, 20])
    frc = np.tile([0.0, 0.0, -1e-4], (6, 1))
    master, _, _ = _setup()
    w16 = torch.zeros(lbm.LBML_NPARAM, dtype=torch.int16, device="cuda")
    lbm.lbml_round_bf16(torch.tensor(master, device="cuda"), w16)
    inv_a, c0, scale, tau = 1 / 0.117, 0.76, 0.01, 0.8
    tr = mobility.Trained(master=None, w16=w16, mu_plain=c0, out_scale=scale, losses=[])
    lat = lbm.Lattice(shape, "fp64", tau=tau, zero_net_force=True, max_points=6)
    dpos = torch.tensor(pos, device="cuda")
    lat.add_point_forces(dpos, torch.tensor(frc, device="cuda"), None, lbm.LB_COLLOIDS, tr.model(inv_a))
    lat.step(80)
    lat.sync()

    def inv_aL_fn(p, t):
        o = p - np.floor(p)
        x = mobility.features(o, np.full(len(p), t))
        y, _ = omlp.forward(master, x)
        return c0 + scale * y

    box = oracle.Box(shape, tau, zero_net_force=True)
    box.sets = [oracle.ForceSet(pos.copy(), frc, kind="colloid", inv_a=inv_a, inv_aL=c0, inv_aL_fn=inv_aL_fn)]
    box.step(80)
    R = dpos.cpu().numpy()
    d = np.abs(R - box.sets[0].pos)
    d = np.minimum(d, np.array([24, 20, 20]) - d)
    disp = np.abs(box.sets[0].pos - pos)
    disp = np.minimum(disp, np.array([24, 20, 20]) - disp).max()
    assert d.max() <= 1e-7 * disp
    # and the correction is not zero: the plain update lands elsewhere
    box2 = oracle.Box(shape, tau, zero_net_force=True)
    box2.sets = [oracle.ForceSet(pos.copy(), frc, kind="colloid", inv_a=inv_a, inv_aL=c0)]
    box2.step(80)
    assert np.abs(box2.sets[0].pos - box.sets[0].pos).max() > 100 * d.max()
