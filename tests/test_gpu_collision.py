"""GPU parity of the general collision operators (Eq. mrtlbe) against the
brute-force FP64 oracle, which builds the 19 x 19 collision matrix explicitly.

* BGK (Eq. bgklbe): every non-conserved mode at 1/tau, ghosts kept;
* MRT: shear modes at 1/tau, the bulk mode at 1/tau_b, all ghosts at one rate;
* with tau_b = tau and ghost rate 2 the MRT path reproduces the projected one.
Bars as in the other parity tests: 1e-10 (FP64 storage), 1e-5 (FP32), relative
to the largest velocity; FP16 storage within the bound of its rounding model.
"""
import numpy as np
import pytest

import oracle
from oracle import bruteforce as bf

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_0707_1299_amd import lbm, workloads  # noqa: E402

TOL = {"fp64": 1e-10, "fp32": 1e-5, "mom32": 1e-5, "fp16": 5e-3}


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def brute_run(shape, tau, tau_b, lam, pos, frc, steps, zero_net=False, colloid=None):
    """Spread (C oracle), literal Eq. mrtlbe collision + propagation (brute force), interpolation
    and, for colloids, the Sec. IV update (C oracle).  Returns (u [3, ...], U at the last step, R)."""
    bb = bf.BruteBox(shape, tau, 1.0, tau_b, lam)
    pos = np.array(pos, dtype=np.float64)
    U = None
    for _ in range(steps):
        g = np.moveaxis(oracle.spread(shape, pos, frc, zero_net), 0, -1)
        _, v = bb.moments(g)
        U = oracle.interp(np.ascontiguousarray(np.moveaxis(v, -1, 0)), pos)
        bb.step(g)
        if colloid:
            pos = oracle.advect(shape, 1.0, tau, pos, frc, U, colloid["inv_a"], colloid["inv_aL"])
    g = np.moveaxis(oracle.spread(shape, pos, frc, zero_net), 0, -1)
    _, v = bb.moments(g)
    return np.moveaxis(v, -1, 0), U, pos


def gpu_run(shape, storage, tau, pos, frc, steps, zero_net=False, colloid=None, nboxes=1, box=None, **coll):
    lat = lbm.Lattice(shape, storage, nboxes=nboxes, tau=tau, zero_net_force=zero_net, max_points=len(pos), **coll)
    p, f = dev(pos), dev(frc)
    vel = torch.zeros_like(p)
    kind = lbm.LB_COLLOIDS if colloid else lbm.LB_FORCES_STATIC
    b = None if box is None else dev(box, torch.int32)
    lat.add_point_forces(p, f, b, kind, lbm.PointModel(vel_out=vel, **(colloid or {})))
    lat.step(steps)
    _, u = lat.moments(rho=False)
    lat.sync()
    return u.cpu().numpy(), vel.cpu().numpy(), p.cpu().numpy()


def _forces(shape, n, seed, scale=1e-5):
    g = np.random.default_rng(seed)
    nz, ny, nx = shape
    pos = g.uniform(0, 1, (n, 3)) * np.array([nx, ny, nz])
    frc = g.normal(scale=scale, size=(n, 3))
    return pos, frc


@pytest.mark.parametrize("storage", ["fp64", "fp32", "fp16"])
def test_bgk_matches_oracle(storage):
    shape = (12, 10, 14)
    tau = 0.8
    pos, frc = _forces(shape, 5, 1)
    u, U, _ = gpu_run(shape, storage, tau, pos, frc, 60, zero_net=True, collision="bgk")
    uo, Uo, _ = brute_run(shape, tau, tau, 1 / tau, pos, frc, 60, zero_net=True)
    e, eU = rel(u[0], uo), rel(U, Uo)
    print("bgk %s: u rel %.3e, U rel %.3e" % (storage, e, eU))
    assert e <= TOL[storage]
    assert eU <= TOL[storage]


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
@pytest.mark.parametrize("rates", [(0.7, 1.6, 1.3), (1.1, 0.6, 0.4), (0.6, 0.6, 3.5)])
def test_mrt_matches_oracle(storage, rates):
    tau, tb, lam = rates
    shape = (10, 12, 16)
    pos, frc = _forces(shape, 6, 2)
    u, U, _ = gpu_run(shape, storage, tau, pos, frc, 50, collision="mrt", tau_bulk=tb, ghost_rate=lam)
    uo, Uo, _ = brute_run(shape, tau, tb, lam, pos, frc, 50)
    e, eU = rel(u[0], uo), rel(U, Uo)
    print("mrt %s %s: u rel %.3e, U rel %.3e" % (storage, rates, e, eU))
    assert e <= TOL[storage]
    assert eU <= TOL[storage]


def test_mrt_with_projected_rates_matches_default_operator():
    shape = (16, 12, 20)
    pos, frc = _forces(shape, 8, 3)
    u0, U0, _ = gpu_run(shape, "fp64", 0.9, pos, frc, 40)
    u1, U1, _ = gpu_run(shape, "fp64", 0.9, pos, frc, 40, collision="mrt", tau_bulk=0.9, ghost_rate=2.0)
    assert rel(u1[0], u0[0]) < 1e-13
    assert rel(U1, U0) < 1e-13


def test_moment_storage_with_bulk_rate():
    """Moment storage holds no ghosts; with them projected out it supports a separate bulk rate."""
    shape = (12, 12, 12)
    pos, frc = _forces(shape, 4, 4)
    u, U, _ = gpu_run(shape, "mom32", 0.6, pos, frc, 50, collision="mrt", tau_bulk=1.4, ghost_rate=2.0)
    uo, Uo, _ = brute_run(shape, 0.6, 1.4, 2.0, pos, frc, 50)
    assert rel(u[0], uo) <= TOL["mom32"]
    assert rel(U, Uo) <= TOL["mom32"]


def test_bgk_colloids_advected():
    shape = (12, 12, 16)
    pos, frc = workloads.colloids(0, 6, shape=shape)
    frc[:, 2] = -1e-4
    model = dict(inv_a=1 / 0.117, inv_aL=0.77)
    u, U, R = gpu_run(shape, "fp64", 0.7, pos, frc, 80, zero_net=True, colloid=model, collision="bgk")
    uo, Uo, Ro = brute_run(shape, 0.7, 0.7, 1 / 0.7, pos, frc, 80, zero_net=True, colloid=model)
    assert rel(u[0], uo) <= TOL["fp64"]
    d = np.abs(R - Ro)
    d = np.minimum(d, np.array([16, 12, 12]) - d)
    disp = np.abs(Ro - pos)
    disp = np.minimum(disp, np.array([16, 12, 12]) - disp).max()
    assert d.max() <= TOL["fp64"] * disp


def test_batched_boxes_with_per_box_rates_equal_single_runs():
    L = 12
    w = workloads.mobility_boxes(nboxes=3, L=L, kmax=2)
    taus = w["taus"]
    tbs = np.array([0.7, 1.9, 0.55])
    ub, Ub, _ = gpu_run((L, L, L), "fp32", taus, w["pos"], w["force"], 40, zero_net=True, nboxes=3, box=w["box"],
                        collision="mrt", tau_bulk=tbs, ghost_rate=1.1)
    for b in range(3):
        m = w["box"] == b
        u1, U1, _ = gpu_run((L, L, L), "fp32", taus[b], w["pos"][m], w["force"][m], 40, zero_net=True,
                            collision="mrt", tau_bulk=tbs[b], ghost_rate=1.1)
        assert np.array_equal(ub[b], u1[0])
        assert np.array_equal(Ub[m], U1)
    m = w["box"] == 1
    uo, _, _ = brute_run((L, L, L), taus[1], tbs[1], 1.1, w["pos"][m], w["force"][m], 40, zero_net=True)
    assert rel(ub[1], uo) <= TOL["fp32"]


def test_bad_tau_bulk_rejected():
    with pytest.raises(lbm.LBError) as e:
        lbm.Lattice((8, 8, 8), "fp32", collision="mrt", tau_bulk=-1.0)
    assert e.value.status == lbm.LB_ERR_ARG
