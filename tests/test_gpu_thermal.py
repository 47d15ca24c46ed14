"""Fluctuating LB and Brownian point colloids on the GPU.

Parity: the thermal step draws the same Philox4x32-10 numbers as the oracle
(counter = node or point index, box, step; key = seed), so the HIP path and
the FP64 oracle follow the same trajectory: bars 1e-10 (FP64) and 1e-5 (FP32)
relative to the largest velocity, as for the deterministic path.

Physics (statistical, fixed seeds):
* equipartition: <j_a^2> = rho kT and <drho^2> = rho kT / cs^2 per node;
* Appendix B: an unforced tracer in the thermal fluid diffuses with
  D = kT mu(L) / (6 pi eta), mu(L) the dimensionless lattice mobility measured
  deterministically (sedimentation) at the same offsets; with the extra noise
  zeta' and 1/a_L set to mu(L), D = kT / (6 pi eta a).
"""
import math

import numpy as np
import pytest

from oracle import fluct

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_0707_1299_amd import lbm, mobility  # noqa: E402

TOL = {"fp64": 1e-10, "fp32": 1e-5}
SEED = 0x1234_5678_9ABC_DEF0


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def gpu_run(shape, storage, tau, kT, steps, sets=(), zero_net=False, step_chunks=None, tile=None, variant=0, **coll):
    npts = sum(len(s["pos"]) for s in sets)
    lat = lbm.Lattice(shape, storage, tau=tau, zero_net_force=zero_net, max_points=max(npts, 1), kT=kT, seed=SEED,
                      tile=tile, variant=variant, **coll)
    outs = []
    for s in sets:
        p, f = dev(s["pos"]), dev(s["force"])
        vel = torch.zeros_like(p)
        if s["kind"] == "colloid":
            m = lbm.PointModel(vel_out=vel, inv_a=s["inv_a"], inv_aL=s["inv_aL"])
            lat.add_point_forces(p, f, None, lbm.LB_COLLOIDS, m)
        else:
            lat.add_point_forces(p, f, None, lbm.LB_FORCES_STATIC, lbm.PointModel(vel_out=vel))
        outs.append((p, vel))
    for n in (step_chunks or [steps]):
        lat.step(n)
    _, u = lat.moments(rho=False)
    lat.sync()
    return u.cpu().numpy()[0], [(p.cpu().numpy(), v.cpu().numpy()) for p, v in outs]


def _sets(shape, seed, colloid=False):
    g = np.random.default_rng(seed)
    nz, ny, nx = shape
    pos = g.uniform(0, 1, (5, 3)) * np.array([nx, ny, nz])
    frc = g.normal(scale=1e-5, size=(5, 3))
    if colloid:
        return [dict(pos=pos, force=frc, kind="colloid", inv_a=1 / 0.117, inv_aL=0.77)]
    return [dict(pos=pos, force=frc, kind="static")]


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
@pytest.mark.parametrize("op", ["projected", "bgk", "mrt"])
def test_thermal_step_matches_oracle(storage, op):
    shape = (8, 6, 10)
    tau, kT = 0.8, 1e-5
    coll = dict(projected=dict(), bgk=dict(collision="bgk"), mrt=dict(collision="mrt", tau_bulk=1.3, ghost_rate=0.9))[op]
    okw = dict(projected=dict(), bgk=dict(ghost_rate=1 / tau), mrt=dict(tau_b=1.3, ghost_rate=0.9))[op]
    sets = _sets(shape, 1)
    u, outs = gpu_run(shape, storage, tau, kT, 30, sets, **coll)
    box = fluct.FluctBox(shape, tau, kT, SEED, sets=sets, **okw)
    box.step(30)
    _, uo = box.moments()
    e, eU = rel(u, uo), rel(outs[0][1], box.sets[0]["U"])
    print("thermal %s %s: u rel %.3e, U rel %.3e (|u| %.2e)" % (op, storage, e, eU, np.abs(uo).max()))
    assert e <= TOL[storage]
    assert eU <= TOL[storage]


def test_brownian_colloids_match_oracle():
    shape = (10, 8, 12)
    tau, kT = 0.7, 1e-5
    sets = _sets(shape, 2, colloid=True)
    u, outs = gpu_run(shape, "fp64", tau, kT, 40, sets, zero_net=True)
    box = fluct.FluctBox(shape, tau, kT, SEED, sets=sets, zero_net=True)
    box.step(40)
    _, uo = box.moments()
    assert rel(u, uo) <= TOL["fp64"]
    R, Ro = outs[0][0], box.sets[0]["pos"]
    d = np.abs(R - Ro)
    d = np.minimum(d, np.array([12, 8, 10]) - d)
    disp = np.abs(Ro - sets[0]["pos"])
    disp = np.minimum(disp, np.array([12, 8, 10]) - disp).max()
    print("brownian colloids: pos err %.3e (disp %.3e)" % (d.max(), disp))
    assert d.max() <= TOL["fp64"] * disp


def test_thermal_run_independent_of_graphs_tiles_and_variants():
    shape = (32, 32, 32)
    sets = _sets(shape, 3, colloid=True)
    u0, o0 = gpu_run(shape, "fp32", 0.6, 1e-5, 41, sets)                                        # graphs + tail
    u1, o1 = gpu_run(shape, "fp32", 0.6, 1e-5, 41, sets, step_chunks=[3] * 13 + [2])            # other split
    u2, o2 = gpu_run(shape, "fp32", 0.6, 1e-5, 41, sets, tile=(32, 4, 2), variant=6)
    u3, o3 = gpu_run(shape, "fp32", 0.6, 1e-5, 41, sets, variant=128)                          # no tile loop
    assert np.array_equal(u0, u1) and np.array_equal(u0, u2) and np.array_equal(u0, u3)
    assert np.array_equal(o0[0][0], o3[0][0])
    assert np.array_equal(o0[0][0], o1[0][0])


@pytest.mark.parametrize("op", ["projected", "bgk"])
def test_equipartition_on_gpu(op):
    L = 32
    kT, tau = 1e-5, 0.8
    coll = dict(collision="bgk") if op == "bgk" else {}
    lat = lbm.Lattice((L, L, L), "fp32", tau=tau, kT=kT, seed=SEED + 1, **coll)
    lat.step(400)
    jj, rr = [], []
    for _ in range(120):
        lat.step(10)
        rho, u = lat.moments()
        j = (rho[0] * u[0]).double()
        jj.append(float((j ** 2).mean()))
        rr.append(float(((rho[0] - 1.0) ** 2).mean()))
    lat.sync()
    N = L ** 3
    jv = np.mean(jj) / (kT * (1 - 1 / N))
    rv = np.mean(rr) / (kT / fluct.CS2 * (1 - 1 / N))
    print("gpu equipartition %s: <j^2>/(rho kT) %.4f, <drho^2>/(rho kT/cs2) %.4f" % (op, jv, rv))
    assert abs(jv - 1) < 0.02
    assert abs(rv - 1) < 0.02


def _msd_D(L, tau, kT, inv_a, inv_aL, nboxes, windows, lag, seed):
    """Diffusion coefficient of one unforced point particle per box: in each window the slope
    (MSD(2 lag) - MSD(lag)) / (6 lag), free of the short-time part of the velocity correlation."""
    g = np.random.default_rng(seed)
    pos = np.full((nboxes, 3), L / 2.0) + g.uniform(0, 1, (nboxes, 3))
    lat = lbm.Lattice((L, L, L), "fp32", nboxes=nboxes, tau=tau, kT=kT, seed=seed, max_points=nboxes)
    p = dev(pos)
    lat.add_point_forces(p, torch.zeros_like(p), dev(np.arange(nboxes), torch.int32), lbm.LB_COLLOIDS,
                         lbm.PointModel(inv_a=inv_a, inv_aL=inv_aL))
    lat.step(2 * L * L)     # momentum diffusion across the box
    est = []

    def disp(a, b):
        d = b - a
        return d - L * np.round(d / L)

    for _ in range(windows):
        p0 = p.cpu().numpy().copy()
        lat.step(lag)
        p1 = p.cpu().numpy().copy()
        lat.step(lag)
        p2 = p.cpu().numpy().copy()
        d1 = disp(p0, p1)
        d2 = d1 + disp(p1, p2)
        est.append(((d2 ** 2).sum(1) - (d1 ** 2).sum(1)) / (6 * lag))
    lat.close()
    est = np.concatenate(est)
    return est.mean(), est.std() / math.sqrt(len(est)), pos - L / 2.0


def test_tracer_diffusion_gives_lattice_mobility():
    """Appendix B: with zeta' off (1/a = 1/a_L) the tracer diffuses as a sphere of radius a_L:
    D 6 pi eta / kT equals the deterministic lattice mobility mu(L) at the same offsets."""
    L, tau, kT = 16, 0.5, 2e-5
    eta = tau / 3
    D, dD, off = _msd_D(L, tau, kT, 1.0 + 1e-12, 1.0, 256, 16, 800, 21)
    mu = mobility.single_particle_labels(off[:64], np.full(64, tau), L=L, steps=1500, average=200)
    got = D * 6 * math.pi * eta / kT
    print("tracer: D 6 pi eta / kT = %.4f +- %.4f, mean mu(L) = %.4f" % (got, dD * 6 * math.pi * eta / kT, mu.mean()))
    assert abs(got / mu.mean() - 1) < 0.06


def test_extra_noise_restores_stokes_einstein_for_radius_a():
    """With 1/a_L = mu(L) the extra displacement zeta' of Appendix B makes D = kT / (6 pi eta a)
    (a in the periodic box, i.e. mu(L) replaced by 1/a)."""
    L, tau, kT = 16, 0.5, 2e-5
    eta = tau / 3
    off = np.random.default_rng(21).uniform(0, 1, (64, 3))
    mu = mobility.single_particle_labels(off, np.full(64, tau), L=L, steps=1500, average=200).mean()
    inv_a = 2.0
    D, dD, _ = _msd_D(L, tau, kT, inv_a, mu, 256, 12, 800, 22)
    got = D * 6 * math.pi * eta / kT
    print("tracer + zeta': D 6 pi eta / kT = %.4f +- %.4f, 1/a = %.4f" % (got, dD * 6 * math.pi * eta / kT, inv_a))
    assert abs(got / inv_a - 1) < 0.06


@pytest.mark.parametrize("shape", [(8, 6, 10), (6, 5, 9)])
def test_fp16_thermal_step_matches_oracle(shape):
    """Scaled FP16 storage with thermal noise: the scale exponent starts from the thermal amplitude
    (no overflow at the first noisy step) and the trajectory follows the oracle's to the FP16 bar
    (5e-3 of the largest velocity); nx = 10 runs two nodes per lane, nx = 9 one."""
    tau, kT = 0.8, 1e-5
    sets = _sets(shape, 4)
    u, outs = gpu_run(shape, "fp16", tau, kT, 30, sets)
    box = fluct.FluctBox(shape, tau, kT, SEED, sets=sets)
    box.step(30)
    _, uo = box.moments()
    e, eU = rel(u, uo), rel(outs[0][1], box.sets[0]["U"])
    print("thermal fp16 %s: u rel %.3e, U rel %.3e" % (shape, e, eU))
    assert e <= 5e-3
    assert eU <= 5e-3
