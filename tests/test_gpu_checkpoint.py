"""Checkpoint and resume: 2n steps in one context equal n steps, a checkpoint,
a new context restored from it and n more steps, bit for bit (velocity field,
colloid positions, interpolated velocities, step count).

Cases: FP32 and FP16-scaled storage with sedimenting colloids fast enough to
leave their binning windows (the restored windows must reproduce the tile
lists of the uninterrupted run), and the fluctuating FP32 step (the thermal
step counter is part of the state).  A checkpoint of another lattice is
rejected.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_0707_1299_amd import lbm, workloads  # noqa: E402

SHAPE = (24, 20, 28)
MODEL = dict(inv_a=1 / 0.117, inv_aL=0.77)


def _lattice(storage, kT):
    return lbm.Lattice(SHAPE, storage, tau=0.7, zero_net_force=True, max_points=12, kT=kT, seed=5,
                       fp16_exponent=12 if storage == "fp16" else 0)


def _register(lat, pos, frc):
    p = torch.tensor(pos, dtype=torch.float64, device="cuda")
    vel = torch.zeros_like(p)
    lat.add_point_forces(p, torch.tensor(frc, dtype=torch.float64, device="cuda"), None, lbm.LB_COLLOIDS,
                         lbm.PointModel(vel_out=vel, **MODEL))
    return p, vel


def _state(lat, p, vel):
    _, u = lat.moments(rho=False)
    lat.sync()
    return u.cpu().numpy(), p.cpu().numpy(), vel.cpu().numpy()


@pytest.mark.parametrize("storage,kT", [("fp32", 0.0), ("fp16", 0.0), ("fp32", 1e-5), ("fp64", 0.0)])
def test_resume_equals_uninterrupted_run(storage, kT):
    pos, frc = workloads.colloids(0, 12, shape=SHAPE)
    frc[:, 2] = -0.01          # about 0.02 nodes per step: the colloids cross their windows
    n = 37
    a = _lattice(storage, kT)
    pa, va = _register(a, pos, frc)
    a.step(2 * n)
    ua, Ra, Ua = _state(a, pa, va)
    a.close()

    b = _lattice(storage, kT)
    pb, vb = _register(b, pos, frc)
    b.step(n)
    buf = torch.empty(b.checkpoint_bytes() + 256, dtype=torch.uint8, device="cuda")
    b.checkpoint_save(buf)
    saved_pos = pb.clone()
    b.sync()
    b.close()

    c = _lattice(storage, kT)
    pc, vc = _register(c, saved_pos.cpu().numpy(), frc)
    c.checkpoint_load(buf)
    assert c.steps_taken() == n
    c.step(n)
    uc, Rc, Uc = _state(c, pc, vc)
    assert c.steps_taken() == 2 * n
    moved = np.abs(Ra - pos).max()
    print("resume %s kT=%g: max displacement %.3f nodes, max |u| %.3e" % (storage, kT, moved, np.abs(ua).max()))
    assert moved > 1.0          # the lists were rebuilt on the way
    assert np.array_equal(ua, uc)
    assert np.array_equal(Ra, Rc)
    assert np.array_equal(Ua, Uc)


def test_checkpoint_of_another_lattice_rejected():
    a = lbm.Lattice((8, 8, 8), "fp32", tau=0.8)
    a.step(3)
    buf = torch.empty(a.checkpoint_bytes() + 256, dtype=torch.uint8, device="cuda")
    a.checkpoint_save(buf)
    a.sync()
    b = lbm.Lattice((8, 8, 12), "fp32", tau=0.8)
    with pytest.raises(lbm.LBError) as e:
        b.checkpoint_load(buf)
    assert e.value.status == lbm.LB_ERR_ARG
    junk = torch.zeros(a.checkpoint_bytes() + 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(lbm.LBError) as e:
        a.checkpoint_load(junk)
    assert e.value.status == lbm.LB_ERR_ARG
