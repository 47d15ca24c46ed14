"""FP16 storage, step kernel with two adjacent x nodes per lane.

With nx even, each lane of the FP16 step kernel takes nodes x and x + 1 with
32-bit accesses; the x-shifted halves come from the neighbouring lane (DPP wave
shift) or, at tile-row and box-row ends, from extra loads.  Variant bit 32
forces one node per lane.  Both do the same arithmetic per node, but the
compiler fuses multiply-adds differently in the two kernels, so single FP32
roundings differ and reach the stored FP16 values as one-ulp differences
(~1.5e-4 of the velocity scale).  The two paths are compared at a bar of 1e-3
relative to the largest value (velocity field, interpolated velocities, moved
colloids, BGK and thermal runs): a wrong shift or edge value would put an
error of order the local velocity at the nodes it touches.  Cases cover every
tile width (waves spanning one row or several), ragged tiles, forces on the
periodic seams and the box-row wrap.  Both paths are also checked against the
FP64 oracle at the FP16 bar.
"""
BAR = 1e-3
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_0707_1299_amd import lbm  # noqa: E402


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def inputs(shape):
    nz, ny, nx = shape
    g = np.random.default_rng(11)
    pos = g.uniform(0, 1, (7, 3)) * np.array([nx, ny, nz])
    pos[0] = [nx - 0.3, 0.2, nz - 0.1]          # on the periodic seams
    pos[1] = [0.05, ny - 0.02, 0.5]
    frc = g.normal(scale=2e-5, size=(7, 3))
    return pos, frc


def run(shape, tile, variant, steps, colloids=False, **kw):
    pos, frc = inputs(shape)
    lat = lbm.Lattice(shape, "fp16", tau=0.8, max_points=7, tile=tile, variant=variant,
                      zero_net_force=colloids, **kw)
    p, f = dev(pos), dev(frc)
    vel = torch.zeros_like(p)
    if colloids:
        lat.add_point_forces(p, f, None, lbm.LB_COLLOIDS, lbm.PointModel(vel_out=vel, inv_a=1 / 0.2, inv_aL=0.77))
    else:
        lat.add_point_forces(p, f, None, lbm.LB_FORCES_STATIC, lbm.PointModel(vel_out=vel))
    lat.step(steps)
    rho, u = lat.moments()
    lat.sync()
    return rho.cpu().numpy(), u.cpu().numpy(), p.cpu().numpy(), vel.cpu().numpy()


CASES = [
    ((13, 10, 70), (128, 2, 1), 0),     # ragged wave: the box row ends inside the wave
    ((13, 10, 70), (32, 4, 2), 0),      # waves over several tile rows, ragged in x
    ((9, 6, 256), (256, 1, 1), 16),     # two waves per tile row, blocks in launch order
    ((12, 12, 128), (128, 1, 2), 2),    # one wave per row, cached loads
    ((10, 8, 64), (64, 2, 2), 4),       # two tiles per block
    ((10, 9, 34), (16, 4, 4), 0),       # 8 lanes per tile row, ragged in every axis
    ((8, 8, 64), (64, 4, 1), 1),        # 64-bit addressing
    ((11, 6, 256), (64, 2, 2), 66),     # the two tiles of a tile row on one XCD, 33 tile rows
    ((9, 7, 512), (128, 2, 1), 82),     # 4 tiles per tile row on one XCD, 36 rows (4 past the last group of 8)
    ((10, 8, 512), (128, 2, 1), 86),    # 2 runs of 2 tiles per tile row on one XCD
    ((13, 10, 70), (128, 2, 1), 128),   # the step kernel without the tile loop, ragged wave
    ((9, 7, 512), (128, 2, 1), 194),    # the same, tile rows on one XCD
]


def report(a, b):
    for name, x, y in zip(("rho", "u", "pos", "U"), a, b):
        d = np.abs(x - y)
        print("  %-3s max|diff| %.3e  max|ref| %.3e  differing %d of %d" % (name, d.max(), np.abs(y).max(),
                                                                          int((d > 0).sum()), d.size), flush=True)


@pytest.mark.parametrize("shape,tile,variant", CASES)
def test_two_nodes_per_lane_match_one(shape, tile, variant):
    a = run(shape, tile, variant, 50)
    b = run(shape, tile, variant | 32, 50)
    report(a, b)
    close(a, b)
    assert np.abs(a[1]).max() > 0


def close(a, b, pos0=None):
    rho_a, u_a, p_a, U_a = a
    rho_b, u_b, p_b, U_b = b
    assert np.abs(u_a - u_b).max() <= BAR * np.abs(u_b).max()
    assert np.abs(rho_a - rho_b).max() <= BAR * np.abs(rho_b - 1.0).max()
    assert np.abs(U_a - U_b).max() <= BAR * np.abs(U_b).max()
    if pos0 is None:
        assert np.array_equal(p_a, p_b)       # static forces: positions untouched
    else:
        disp = np.abs(p_b - pos0).max()
        assert np.abs(p_a - p_b).max() <= BAR * max(disp, 1e-30)


@pytest.mark.parametrize("shape,tile,variant", [((13, 10, 70), (128, 2, 1), 0), ((13, 10, 70), (128, 2, 1), 32),
                                                ((10, 9, 34), (16, 4, 4), 0), ((9, 6, 256), (256, 1, 1), 16)])
def test_fp16_paths_against_oracle(shape, tile, variant):
    """Both FP16 step paths against the FP64 oracle on ragged boxes with seam forces."""
    import oracle
    pos, frc = inputs(shape)
    _, u, _, U = run(shape, tile, variant, 50)
    box = oracle.Box(shape, 0.8, 1.0)
    box.sets = [oracle.ForceSet(pos, frc, kind="static")]
    box.step(50)
    _, uo = box.moments()
    e = float(np.abs(u[0] - uo).max() / np.abs(uo).max())
    eU = float(np.abs(U - box.sets[0].U).max() / np.abs(box.sets[0].U).max())
    print("fp16 %s %s variant %d vs oracle: u rel %.3e, U rel %.3e" % (shape, tile, variant, e, eU), flush=True)
    assert e <= 5e-3 and eU <= 5e-3


@pytest.mark.parametrize("shape,tile", [((13, 10, 70), (128, 2, 1)), ((10, 9, 34), (32, 2, 4))])
def test_two_nodes_per_lane_colloids_bgk_thermal(shape, tile):
    pos0 = inputs(shape)[0]
    for kw in (dict(), dict(collision="bgk"), dict(kT=1e-6, seed=3)):
        a = run(shape, tile, 0, 40, colloids=True, **kw)
        b = run(shape, tile, 32, 40, colloids=True, **kw)
        print(kw)
        report(a, b)
        close(a, b, pos0)
