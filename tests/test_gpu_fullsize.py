"""The benchmark workloads at their full sizes and stated run lengths, against the
FP64 oracle, in the launch configuration the benchmark times (tuned tile and
access variant, graph replay):

* 128^3 singularities (64 multipoles, 149 point forces), FP32, the full 5000
  steps;
* 256^3 with 10^4 sedimenting colloids (a = 0.117), FP64, FP32 and FP16-scaled
  storage, 1000 steps, each against one oracle run and against the FP64 GPU
  run, with the total mass and momentum of every storage (Eq. conservation);
* 512 independent 32^3 boxes (1-8 fixed colloids each, tau_b ~ U[0.6, 1.5]),
  FP32 and FP16, the full 2000 steps with the interpolated velocity averaged
  over the last 200, four boxes checked against one-box oracle runs;
* 512^3 with 10^5 colloids (a = 0.684): plain FP32 against the oracle with the
  same constant 1/a_L, and FP16 with the trained mobility network against the
  oracle evaluating the same bf16 network in FP64, 10 steps each.

The two long single-lattice runs are compared with the oracle's results
sampled by tests/golden/make_long_goldens.py (it calls only the oracle; a run
takes an hour on the host): the velocity at the 2x2x2 nodes around the force
points (or 512 colloids) and at 2048 uniform nodes, the interpolated velocity
and positions of the points, and the population sums.  The norm is the one of
the smaller parity tests: max |u - u_oracle| over the sampled nodes and
components divided by max |u_oracle| over the whole lattice (stored with the
samples); interpolated velocities likewise; position errors relative to the
oracle's displacement.  Bars: 1e-10 (FP64), 1e-5 (FP32) and the FP16 rounding
bound 5e-3.
"""
import hashlib
import os

import numpy as np
import pytest

import oracle
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_0707_1299_amd import lbm, mobility, tune, workloads  # noqa: E402

TOL = {"fp64": 1e-10, "fp32": 1e-5, "fp16": 5e-3}
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def golden(name):
    d = dict(np.load(os.path.join(GOLDEN, name), allow_pickle=False))
    sha = hashlib.sha256(open(os.path.join(ROOT, "oracle", "lbm_oracle.c"), "rb").read()).hexdigest()
    assert str(d["oracle_sha"]) == sha, "%s was written by another oracle source: rerun make_long_goldens.py" % name
    return d


def wrap_err(a, b, ext):
    d = np.abs(a - b)
    return np.minimum(d, ext - d)


def lattice(shape, storage, tag, **kw):
    tile, variant = tune.lookup(shape, storage, kw.get("nboxes", 1), tag) or (None, 0)
    print("%s %s: tile %s variant %d" % (tag, storage, tile, variant), flush=True)
    return lbm.Lattice(shape, storage, tile=tile, variant=variant, **kw)


def test_singularities128_fp32_5000_steps():
    d = golden("singularities128_oracle_5000.npz")
    L = 128
    w = workloads.singularities(L=L, n=64)
    pos, frc = lbm.lb_expand_multipoles(w["types"], w["centers"], w["axes"], w["e1"], w["strengths"], w["sep"])
    assert np.array_equal(pos, d["pos"])
    lat = lattice((L, L, L), "fp32", "singularities128", tau=0.5, max_points=len(pos))
    p = torch.tensor(pos, device="cuda")
    vel = torch.zeros_like(p)
    lat.add_point_forces(p, torch.tensor(frc, device="cuda"), None, lbm.LB_FORCES_STATIC,
                         lbm.PointModel(vel_out=vel))
    lat.step(int(d["steps"]))
    _, u = lat.moments(rho=False)
    lat.sync()
    us = u[0].reshape(3, -1)[:, torch.tensor(d["nodes"], device="cuda")].cpu().numpy()
    e = float(np.abs(us - d["u"]).max() / d["umax"])
    eU = rel(vel.cpu().numpy(), d["U"])
    print("128^3 fp32 after %d steps: u rel %.3e (%d sampled nodes), U rel %.3e"
          % (int(d["steps"]), e, len(d["nodes"]), eU), flush=True)
    assert e <= TOL["fp32"]
    assert eU <= TOL["fp32"]


@pytest.fixture(scope="module")
def colloids256():
    """One 1000-step run per storage of the 256^3 colloid workload: sampled fields, the sampled
    colloids, diagnostics and the full velocity field (kept for the cross-storage comparison)."""
    d = golden("colloids256_oracle_1000.npz")
    L, n = 256, 10000
    pos, frc = workloads.colloids(L, n)
    assert np.array_equal(pos[d["pick"]], d["pos0"])
    out = {}
    nodes = torch.tensor(d["nodes"], device="cuda")
    for st in ("fp64", "fp32", "fp16"):
        lat = lattice((L, L, L), st, "colloids256_" + st, tau=0.5, zero_net_force=True, max_points=n)
        p = torch.tensor(pos, device="cuda")
        vel = torch.zeros_like(p)
        lat.add_point_forces(p, torch.tensor(frc, device="cuda"), None, lbm.LB_COLLOIDS,
                             lbm.PointModel(vel_out=vel, inv_a=1 / 0.117, inv_aL=0.77))
        lat.step(int(d["steps"]))
        r, diag = lat.diagnostics()
        assert r == lbm.LB_OK
        rho, u = lat.moments()
        lat.sync()
        out[st] = dict(u=u[0].reshape(3, -1)[:, nodes].cpu().numpy(), ufull=u[0].cpu().numpy(),
                       drho=(rho[0] - 1.0).cpu().numpy(), R=p.cpu().numpy()[d["pick"]],
                       U=vel.cpu().numpy()[d["pick"]], diag=diag[0])
        del u, rho
        lat.close()
        torch.cuda.empty_cache()
        print("256^3 %s: 1000 steps done" % st, flush=True)
    return d, pos, out


@pytest.mark.parametrize("storage", ["fp64", "fp32", "fp16"])
def test_colloids256_1000_steps_against_oracle(colloids256, storage):
    d, pos, out = colloids256
    o = out[storage]
    e = float(np.abs(o["u"] - d["u"]).max() / d["umax"])
    eU = rel(o["U"], d["U"])
    disp = wrap_err(d["pos"], d["pos0"], 256.0).max()
    eR = wrap_err(o["R"], d["pos"], 256.0).max() / disp
    print("256^3 %s vs oracle after 1000 steps: u rel %.3e, U rel %.3e, pos err/disp %.3e (disp %.3e)"
          % (storage, e, eU, eR, disp), flush=True)
    assert e <= TOL[storage]
    assert eU <= TOL[storage]
    assert eR <= TOL[storage]


@pytest.mark.parametrize("storage", ["fp32", "fp16"])
def test_colloids256_1000_steps_against_fp64_gpu(colloids256, storage):
    """The whole velocity field of each reduced storage against the FP64 run of the library."""
    _, _, out = colloids256
    e = rel(out[storage]["ufull"], out["fp64"]["ufull"])
    print("256^3 %s vs FP64 GPU after 1000 steps: u rel %.3e (whole field)" % (storage, e), flush=True)
    assert e <= TOL[storage]


# Storing deviations in a floating-point format conserves neither mass nor momentum exactly: every
# population is rounded each step.  Round-to-nearest of values whose density falls off with their
# magnitude is biased slightly toward zero, and since positive and negative deviations do not balance
# population by population the totals drift roughly linearly in the number of steps (FP32 storage
# shows the same drift, about 2^11 times smaller).  Stated bounds for FP16-scaled storage after
# 1000 steps at 256^3 with 10^4 colloids (counter-force on, so the exact totals stay zero): mass,
# |sum drho| <= 1e-2 of sum |drho| of the FP64 run; momentum, |sum jbar| <= 1e-4 of the momentum the
# colloid forces put in, steps * sum |F|.
FP16_MASS_BOUND, FP16_MOMENTUM_BOUND = 1e-2, 1e-4


def test_colloids256_mass_and_momentum_every_storage(colloids256):
    """Total mass and auxiliary momentum (diagnostics 0-3) of every storage against the oracle's
    population sums and against the FP64 GPU run; FP64 and FP32 at their bars, FP16 at the
    stated bounds."""
    d, _, out = colloids256
    orc_mass = float(d["df_sum"].sum())
    orc_mom = d["c"].T.astype(np.float64) @ d["df_sum"]
    scale_mass = float(np.abs(out["fp64"]["drho"]).sum())
    scale_mom = int(d["steps"]) * 10000 * 1e-6
    for st in ("fp64", "fp32", "fp16"):
        dg = out[st]["diag"]
        em = abs(dg[0] - orc_mass) / scale_mass
        ep = float(np.abs(dg[1:4] - orc_mom).max()) / scale_mom
        em64 = abs(dg[0] - out["fp64"]["diag"][0]) / scale_mass
        ep64 = float(np.abs(dg[1:4] - out["fp64"]["diag"][1:4]).max()) / scale_mom
        print("256^3 %s totals after 1000 steps: mass %.3e (oracle %.3e) -> err %.3e of sum|drho| (vs FP64 GPU "
              "%.3e); momentum %s (oracle %s) -> err %.3e of n sum|F| (vs FP64 GPU %.3e)"
              % (st, dg[0], orc_mass, em, em64, np.array2string(dg[1:4], precision=3),
                 np.array2string(orc_mom, precision=3), ep, ep64), flush=True)
        assert dg[11] == 0 and dg[12] == 0
        if st == "fp16":
            assert em <= FP16_MASS_BOUND and em64 <= FP16_MASS_BOUND
            assert ep <= FP16_MOMENTUM_BOUND and ep64 <= FP16_MOMENTUM_BOUND
        else:
            assert em <= TOL[st] and ep <= TOL[st]


@pytest.mark.parametrize("storage", ["fp32", "fp16"])
def test_boxes512x32_2000_steps_spot_checked(storage):
    """The batched mobility workload as the benchmark runs it: 512 boxes, 2000 steps, the
    interpolated velocity summed over the last 200; four boxes (most colloids, smallest and
    largest tau, one more) against one-box oracle runs of the same steps."""
    w = workloads.mobility_boxes(nboxes=512, L=32)
    nb, steps, avg = 512, 2000, 200
    lat = lattice((32, 32, 32), storage, "boxes512x32_" + storage, nboxes=nb, tau=w["taus"], zero_net_force=True,
                  max_points=len(w["pos"]))
    p = torch.tensor(w["pos"], device="cuda")
    vsum = torch.zeros_like(p)
    lat.add_point_forces(p, torch.tensor(w["force"], device="cuda"), torch.tensor(w["box"], device="cuda"),
                         lbm.LB_FORCES_STATIC, lbm.PointModel(vel_sum=vsum))
    lat.step(steps - avg)
    vsum.zero_()
    lat.step(avg)
    _, u = lat.moments(rho=False)
    lat.sync()
    Ubar = vsum.cpu().numpy() / avg
    check = sorted({int(np.argmax(w["counts"])), int(np.argmin(w["taus"])), int(np.argmax(w["taus"])), 101})
    tol = TOL[storage]
    for b in check:
        m = w["box"] == b
        box = oracle.Box((32, 32, 32), float(w["taus"][b]), 1.0, zero_net_force=True)
        box.sets = [oracle.ForceSet(w["pos"][m].copy(), w["force"][m].copy())]
        box.step(steps - avg)
        Uo = np.zeros((int(m.sum()), 3))
        for _ in range(avg):
            box.step(1)
            Uo += box.sets[0].U
        Uo /= avg
        _, uo = box.moments()
        e = rel(u[b].cpu().numpy(), uo)
        eU = rel(Ubar[m], Uo)
        print("boxes %s box %d (%d colloids, tau %.3f): u rel %.3e, mean U rel %.3e"
              % (storage, b, int(m.sum()), w["taus"][b], e, eU), flush=True)
        assert e <= tol
        assert eU <= tol


def _c5_gpu(storage, model, steps):
    L, n = 512, 100000
    pos, frc = workloads.colloids(L, n)
    lat = lattice((L, L, L), storage, "colloids512_" + storage, tau=0.5, zero_net_force=True, max_points=n)
    p = torch.tensor(pos, device="cuda")
    vel = torch.zeros_like(p)
    model.vel_out = vel
    lat.add_point_forces(p, torch.tensor(frc, device="cuda"), None, lbm.LB_COLLOIDS, model)
    lat.step(steps)
    _, u = lat.moments(rho=False)
    lat.sync()
    res = (u[0].cpu().numpy(), p.cpu().numpy(), vel.cpu().numpy())
    del u
    lat.close()
    torch.cuda.empty_cache()
    print("512^3 %s: %d steps on the GPU done" % (storage, steps), flush=True)
    return res


def _c5_oracle(steps, inv_a, inv_aL, inv_aL_fn=None):
    L, n = 512, 100000
    pos, frc = workloads.colloids(L, n)
    box = oracle.Box((L, L, L), 0.5, 1.0, zero_net_force=True)
    box.sets = [oracle.ForceSet(pos.copy(), frc.copy(), kind="colloid", inv_a=inv_a, inv_aL=inv_aL,
                                inv_aL_fn=inv_aL_fn)]
    box.step(steps)
    _, uo = box.moments()
    print("512^3 oracle: %d steps done" % steps, flush=True)
    return pos, uo, box.sets[0].pos.copy(), box.sets[0].U.copy()


def _c5_compare(name, gpu, orc, tol):
    ug, Rg, Ug = gpu
    pos, uo, Ro, Uo = orc
    disp = wrap_err(Ro, pos, 512.0).max()
    e, eU, eR = rel(ug, uo), rel(Ug, Uo), wrap_err(Rg, Ro, 512.0).max() / disp
    print("512^3 %s vs oracle: u rel %.3e, U rel %.3e, pos err/disp %.3e (disp %.3e)" % (name, e, eU, eR, disp),
          flush=True)
    assert e <= tol
    assert eU <= tol
    assert eR <= tol


def test_colloids512_plain_fp32_10_steps():
    """The plain form of the headline workload: FP32 storage, the constant 1/a_L fitted for tau = 1/2."""
    tr = mobility.load(mobility.DEFAULT_NET)
    inv_a, c = 1 / 0.684, float(tr.plain_tau(0.5))
    gpu = _c5_gpu("fp32", lbm.PointModel(inv_a=inv_a, inv_aL=c), 10)
    _c5_compare("fp32 plain", gpu, _c5_oracle(10, inv_a, c), TOL["fp32"])


def test_colloids512_fp16_with_trained_network_10_steps():
    """The chosen form of the headline workload: FP16-scaled storage and the trained network (the
    file the benchmark loads) in the colloid update; the oracle evaluates the same bf16 weights
    in FP64 for every colloid at every step."""
    tr = mobility.load(mobility.DEFAULT_NET)
    inv_a = 1 / 0.684
    gpu = _c5_gpu("fp16", tr.model(inv_a), 10)
    theta = mobility.weights_f64(tr)

    def inv_aL_fn(p, t):
        o = p - np.floor(p)
        y, _ = omlp.forward(theta, mobility.features(o, np.full(len(p), t)), round_bf16=False)
        return tr.mu_plain + tr.out_scale * y

    _c5_compare("fp16 + MLP", gpu, _c5_oracle(10, inv_a, tr.mu_plain, inv_aL_fn), TOL["fp16"])
