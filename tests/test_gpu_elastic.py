"""Curves and surfaces of singular forces on the GPU against the FP64 oracle.

Markers of bead-spring chains and of a closed triangulated interface get their
forces from their configuration every step, spread them, and move with the
interpolated fluid velocity.  Parity bars as for point forces: 1e-10 (FP64),
1e-5 (FP32) relative to the largest velocity, marker positions relative to
their displacement.  Physics: the Laplace pressure jump 2 gamma / R of a
droplet, and batched boxes equal to single runs bit for bit.
"""
import numpy as np
import pytest

from oracle import elastic

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_0707_1299_amd import lbm  # noqa: E402

TOL = {"fp64": 1e-10, "fp32": 1e-5}


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def chains(shape, nchain, m, seed):
    g = np.random.default_rng(seed)
    nz, ny, nx = shape
    out = []
    for _ in range(nchain):
        start = g.uniform(0, 1, 3) * np.array([nx, ny, nz])
        step = g.normal(size=3)
        step *= 1.4 / np.linalg.norm(step)
        out.append(start + np.arange(m)[:, None] * step + g.normal(scale=0.2, size=(m, 3)))
    pos = np.concatenate(out)
    return pos - np.array([nx, ny, nz]) * np.floor(pos / np.array([nx, ny, nz]))


def ellipsoid(center, radii, levels):
    V, T = elastic.icosphere(np.zeros(3), 1.0, levels)
    return V * np.asarray(radii) + np.asarray(center), T


def run_gpu(shape, storage, tau, steps, chain=None, surf=None, nboxes=1, box=None):
    npts = (len(chain["pos"]) if chain else 0) + (len(surf["pos"]) if surf else 0)
    lat = lbm.Lattice(shape, storage, tau=tau, max_points=npts, nboxes=nboxes)
    out = {}
    if chain:
        p = dev(chain["pos"])
        v = torch.zeros_like(p)
        ext = None if chain.get("ext") is None else dev(chain["ext"])
        b = None if box is None else dev(box, torch.int32)
        lat.add_chains(p, chain["chain_len"], chain["k"], chain["l0"], ext=ext, box=b, vel_out=v)
        out["chain"] = (p, v)
    if surf:
        p = dev(surf["pos"])
        v = torch.zeros_like(p)
        b = None if box is None else dev(box, torch.int32)
        lat.add_surface(p, surf["tri"], surf["tension"], box=b, vel_out=v)
        out["surf"] = (p, v)
    lat.step(steps)
    rho, u = lat.moments()
    lat.sync()
    return rho.cpu().numpy(), u.cpu().numpy(), {k: (p.cpu().numpy(), v.cpu().numpy()) for k, (p, v) in out.items()}


def pos_err(R, Ro, R0, dims):
    d = np.abs(R - Ro)
    d = np.minimum(d, dims - d)
    disp = np.abs(Ro - R0)
    disp = np.minimum(disp, dims - disp).max()
    return d.max(), disp


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
def test_sedimenting_chains_match_oracle(storage):
    shape = (20, 16, 24)
    pos = chains(shape, 3, 8, 5)
    ext = np.tile([0.0, 0.0, -2e-5], (len(pos), 1))
    ch = dict(pos=pos, kind="chain", chain_len=8, k=2e-3, l0=1.0, ext=ext)
    _, u, out = run_gpu(shape, storage, 0.7, 120, chain=ch)
    box = elastic.ElasticBox(shape, 0.7, sets=[ch])
    box.step(120)
    _, uo = box.moments()
    e = rel(u[0], uo)
    d, disp = pos_err(out["chain"][0], box.sets[0]["pos"], pos, np.array([24, 16, 20]))
    print("chains %s: u rel %.3e, pos err %.3e (disp %.3e)" % (storage, e, d, disp))
    assert e <= TOL[storage]
    assert d <= TOL[storage] * disp
    assert rel(out["chain"][1], box.sets[0]["U"]) <= TOL[storage]


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
def test_relaxing_droplet_matches_oracle(storage):
    shape = (24, 20, 22)
    V, T = ellipsoid((11.3, 10.2, 12.1), (5.0, 4.0, 3.5), 2)
    sf = dict(pos=V, kind="surface", tri=T, tension=5e-4)
    _, u, out = run_gpu(shape, storage, 0.8, 150, surf=sf)
    box = elastic.ElasticBox(shape, 0.8, sets=[sf])
    box.step(150)
    _, uo = box.moments()
    e = rel(u[0], uo)
    d, disp = pos_err(out["surf"][0], box.sets[0]["pos"], V, np.array([22, 20, 24]))
    print("droplet %s: u rel %.3e, pos err %.3e (disp %.3e)" % (storage, e, d, disp))
    assert e <= TOL[storage]
    assert d <= TOL[storage] * disp


def test_laplace_pressure_on_gpu():
    L, R, gam, tau = 48, 10.0, 2e-4, 0.8
    c = np.full(3, L / 2 + 0.3)
    V, T = elastic.icosphere(c, R, 4)
    rho, u, _ = run_gpu((L, L, L), "fp32", tau, 4000, surf=dict(pos=V, tri=T, tension=gam))
    z, y, x = np.meshgrid(np.arange(L), np.arange(L), np.arange(L), indexing="ij")
    r = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
    dp = (rho[0][r < R - 3].mean() - rho[0][r > R + 4].mean()) / 3.0
    print("gpu Laplace: c_s^2 drho = %.4e, 2 gamma / R = %.4e, max |u| %.2e" % (dp, 2 * gam / R, np.abs(u).max()))
    assert abs(dp / (2 * gam / R) - 1) < 0.02


def test_batched_boxes_equal_single_runs():
    shape = (16, 16, 16)
    V, T = ellipsoid((8.2, 7.9, 8.4), (4.0, 3.5, 3.0), 2)
    pos2 = np.concatenate([V, V + 0.37])
    tri2 = np.concatenate([T, T + len(V)])
    box = np.repeat([0, 1], len(V))
    _, ub, ob = run_gpu(shape, "fp32", 0.7, 60, surf=dict(pos=pos2, tri=tri2, tension=4e-4), nboxes=2, box=box)
    for b, P in ((0, V), (1, V + 0.37)):
        _, u1, o1 = run_gpu(shape, "fp32", 0.7, 60, surf=dict(pos=P, tri=T, tension=4e-4))
        assert np.array_equal(ub[b], u1[0])
        assert np.array_equal(ob["surf"][0][box == b], o1["surf"][0])


def test_bad_elastic_sets_rejected():
    lat = lbm.Lattice((8, 8, 8), "fp32", max_points=10)
    p = dev(np.ones((6, 3)))
    with pytest.raises(lbm.LBError):
        lat.add_chains(p, 4, 1.0, 1.0)          # 6 markers are not whole chains of 4
    with pytest.raises(lbm.LBError):
        lat.add_chains(p, 1, 1.0, 1.0)
    with pytest.raises(lbm.LBError):
        lat.add_chains(dev(np.ones((12, 3))), 2, 1.0, 1.0)   # beyond max_points
