"""Pins for the curve and surface force oracle (singular forces on markers).

* surface forces are -gamma times the exact gradient of the triangulated area
  (central differences), sum to zero and exert no torque; on a closed surface
  sum_v F_v.(R_v - c) = -2 gamma A exactly (area is homogeneous of degree 2);
* chain springs are internal (zero sum, zero torque), vanish at rest length and
  have magnitude k (r - l0);
* a triangulated droplet of tension gamma in the oracle's fluid develops the
  Laplace pressure jump c_s^2 (rho_in - rho_out) = 2 gamma / R.
"""
import numpy as np
import pytest

from oracle import elastic


def test_surface_force_is_minus_tension_times_area_gradient():
    V, T = elastic.icosphere((10.0, 11.0, 9.0), 4.0, 2)
    rng = np.random.default_rng(3)
    V = V + rng.normal(scale=0.2, size=V.shape)
    L = (40, 40, 40)
    gam = 0.7
    F = elastic.surface_forces(V, T, gam, L)
    h = 1e-6
    for v in rng.choice(len(V), 12, replace=False):
        for a in range(3):
            Vp, Vm = V.copy(), V.copy()
            Vp[v, a] += h
            Vm[v, a] -= h
            fd = (elastic.surface_area(Vp, T, L) - elastic.surface_area(Vm, T, L)) / (2 * h)
            assert abs(-gam * fd - F[v, a]) < 1e-7     # rounding of the area (~200) over 2h


def test_surface_forces_sum_and_torque_vanish_and_virial():
    c = np.array([12.0, 12.0, 12.0])
    V, T = elastic.icosphere(c, 5.0, 3)
    V = V + np.random.default_rng(4).normal(scale=0.1, size=V.shape)
    gam = 1.3
    F = elastic.surface_forces(V, T, gam, (48, 48, 48))
    scale = np.abs(F).max()
    assert np.abs(F.sum(0)).max() < 1e-13 * scale * len(V)
    assert np.abs(np.cross(V - c, F).sum(0)).max() < 1e-12 * scale * len(V)
    A = elastic.surface_area(V, T, (48, 48, 48))
    assert abs((F * (V - c)).sum() + 2 * gam * A) < 1e-12 * gam * A


def test_icosphere_is_closed_and_outward():
    V, T = elastic.icosphere((0.0, 0.0, 0.0), 1.0, 2)
    assert len(V) == 162 and len(T) == 320
    edges = {}
    for t in T:
        for a, b in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0])):
            edges[(a, b)] = edges.get((a, b), 0) + 1
    assert all(edges.get((b, a), 0) == 1 for (a, b) in edges)     # every directed edge has its reverse once
    n = np.cross(V[T[:, 1]] - V[T[:, 0]], V[T[:, 2]] - V[T[:, 0]])
    assert np.all((n * V[T].mean(1)).sum(1) > 0)


def test_chain_springs():
    L = (30, 30, 30)
    pos = np.array([[1.0, 2, 3], [2.5, 2, 3], [2.5, 4, 3], [10, 10, 10], [11, 10, 10]])
    F = elastic.chain_forces(pos, 3, 0.2, 1.0, L)
    assert np.abs(F.sum(0)).max() < 1e-16
    assert np.abs(np.cross(pos, F).sum(0)).max() < 1e-14
    assert np.allclose(F[0], [0.2 * 0.5, 0, 0]) and np.allclose(F[2], [0, -0.2 * 1.0, 0])
    assert np.allclose(F[3:], 0.0)                       # second chain (markers 3, 4) is at rest length
    F2 = elastic.chain_forces(pos[:2], 2, 0.2, 1.5, L)
    assert np.allclose(F2, 0.0)
    # across the periodic seam: minimum image
    F3 = elastic.chain_forces(np.array([[29.5, 1, 1], [0.5, 1, 1]]), 2, 1.0, 0.5, L)
    assert np.allclose(F3[0], [0.5, 0, 0])


def test_laplace_pressure_of_a_droplet():
    L, R, gam, tau = 24, 5.0, 2e-4, 0.8
    c = np.full(3, L / 2 + 0.3)
    V, T = elastic.icosphere(c, R, 3)
    box = elastic.ElasticBox((L, L, L), tau, sets=[dict(pos=V, kind="surface", tri=T, tension=gam)])
    box.step(1500)
    rho, u = box.moments()
    z, y, x = np.meshgrid(np.arange(L), np.arange(L), np.arange(L), indexing="ij")
    r = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
    dp = (rho[r < R - 2.5].mean() - rho[r > R + 3].mean()) / 3.0
    print("Laplace: c_s^2 drho = %.4e, 2 gamma / R = %.4e, max |u| %.2e" % (dp, 2 * gam / R, np.abs(u).max()))
    assert abs(dp / (2 * gam / R) - 1) < 0.1
    assert np.abs(u).max() < 1e-3 * gam / (tau / 3)     # spurious currents small against gamma / eta
