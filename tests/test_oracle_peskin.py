"""Pins for the oracle's regularised delta (Eq. deltadef, Sec. III).

Peskin's 4-point kernel is constructed so that, for any offset, its samples on
the integers sum to 1, have zero first moment, sum of squares 3/8, and equal
even and odd sums.  Its values at half-integers have closed forms
(tests/golden/peskin_values.txt).  The three-dimensional spreading of a unit
force must reproduce the product of one-dimensional transforms exactly.
"""
import os

import numpy as np
import pytest

import oracle
from oracle import analytic, bruteforce

GOLD = os.path.join(os.path.dirname(__file__), "golden", "peskin_values.txt")


def _golden():
    rows = []
    for line in open(GOLD):
        line = line.strip()
        if line and not line.startswith("#"):
            r, v = line.split()[:2]
            rows.append((float(r), float(v)))
    return rows


@pytest.mark.parametrize("r,v", _golden())
def test_phi_closed_form_values(r, v):
    assert oracle.phi(r) == pytest.approx(v, abs=1e-15)
    assert bruteforce.peskin_1d(r) == pytest.approx(v, abs=1e-15)


def test_phi_continuous_at_branch_points():
    for r0 in (1.0, 2.0):
        lo, hi = oracle.phi(r0 - 1e-12), oracle.phi(r0 + 1e-12)
        assert abs(lo - hi) < 1e-9


@pytest.mark.parametrize("frac", np.linspace(0.0, 0.999, 37))
def test_phi_moment_identities(frac):
    R = 7.0 + frac
    nodes = np.arange(3, 12)
    w = np.array([oracle.phi(x - R) for x in nodes])
    assert w.sum() == pytest.approx(1.0, abs=1e-14)
    assert ((nodes - R) * w).sum() == pytest.approx(0.0, abs=1e-14)
    assert (w * w).sum() == pytest.approx(3.0 / 8.0, abs=1e-14)
    even = w[nodes % 2 == 0].sum()
    odd = w[nodes % 2 == 1].sum()
    assert even == pytest.approx(0.5, abs=1e-14)
    assert odd == pytest.approx(0.5, abs=1e-14)
    assert np.count_nonzero(w) <= 4


def test_spread_unit_force_matches_product_transform():
    rng = np.random.default_rng(3)
    shape = (8, 6, 10)
    for _ in range(4):
        R = rng.uniform(-3, 13, size=3)          # outside the box too: wrapped periodically
        g = oracle.spread(shape, R[None], np.array([[1.0, 0.0, 0.0]]))
        G = np.fft.fftn(g[0])
        ref = analytic.peskin_dft(shape, R)
        assert np.abs(G - ref).max() < 1e-14


def test_spread_matches_dense_minimum_image():
    rng = np.random.default_rng(4)
    shape = (5, 4, 7)
    pos = rng.uniform(0, 7, size=(6, 3))
    F = rng.normal(size=(6, 3))
    for zero_net in (False, True):
        g = oracle.spread(shape, pos, F, zero_net)
        gd = bruteforce.spread_dense(shape, pos, F, zero_net)
        assert np.abs(np.moveaxis(g, 0, -1) - gd).max() < 1e-14


def test_spread_force_and_first_moment():
    """sum_x g = F and sum_x x g = R F for a force away from the periodic seam."""
    rng = np.random.default_rng(5)
    shape = (12, 12, 12)
    for _ in range(5):
        R = rng.uniform(3, 8, size=3)
        F = rng.normal(size=3)
        g = oracle.spread(shape, R[None], F[None])
        z, y, x = np.meshgrid(*(np.arange(12),) * 3, indexing="ij")
        assert np.allclose(g.sum((1, 2, 3)), F, atol=1e-14)
        first = np.array([(g[c] * X).sum() for c in range(3) for X in (x, y, z)]).reshape(3, 3)
        assert np.allclose(first, np.outer(F, R), atol=1e-13)


def test_interp_is_adjoint_of_spread():
    """<u, spread(F at R)> = F . interp(u at R): both use the same kernel weights."""
    rng = np.random.default_rng(6)
    shape = (6, 5, 7)
    u = rng.normal(size=(3,) + shape)
    R = rng.uniform(0, 7, size=(4, 3))
    F = rng.normal(size=(4, 3))
    lhs = (u * oracle.spread(shape, R, F)).sum()
    rhs = (F * oracle.interp(u, R)).sum()
    assert lhs == pytest.approx(rhs, rel=1e-13)
    U = oracle.interp(u, R)
    Ud = bruteforce.interp_dense(np.moveaxis(u, 0, -1), R)
    assert np.abs(U - Ud).max() < 1e-13


def test_interp_reproduces_linear_fields():
    """The kernel's zeroth and first moments make interpolation exact for linear fields
    (away from the periodic seam)."""
    shape = (16, 16, 16)
    z, y, x = np.meshgrid(*(np.arange(16.0),) * 3, indexing="ij")
    u = np.stack([0.3 + 0.01 * x - 0.02 * y, 0.05 * z, -0.1 + 0.0 * x])
    R = np.array([[6.3, 7.9, 8.25], [5.5, 5.0, 9.99]])
    U = oracle.interp(u, R)
    exp = np.stack([0.3 + 0.01 * R[:, 0] - 0.02 * R[:, 1], 0.05 * R[:, 2], -0.1 + 0 * R[:, 0]], 1)
    assert np.abs(U - exp).max() < 1e-13


def test_deltaapprox_transform_by_quadrature():
    """Eq. deltaFT is the continuous Fourier transform (k in cycles) of Eq. deltaapprox."""
    r = np.linspace(-2, 2, 40001)
    f = analytic.deltaapprox(r)
    for k in (0.0, 0.1, 0.25, 0.37, 0.5, 1.3):
        num = np.trapezoid(f * np.cos(2 * np.pi * k * r), r)
        assert num == pytest.approx(float(analytic.deltaapprox_ft(k)), abs=1e-7)
    # and it approximates the Peskin kernel to within 0.02 everywhere on the support
    assert np.abs(analytic.deltaapprox(r) - bruteforce.peskin_1d(r)).max() < 0.02
