"""Pins for the fluctuating-LB oracle (thermal noise and Brownian colloids).

* Philox4x32-10 reproduces the published known-answer vectors;
* Box-Muller normals have mean 0, variance 1, kurtosis 3;
* the fifteen mode polynomials are w-orthogonal to each other and to 1, c;
* the node noise changes neither mass nor momentum (exactly, per node) and its
  mode covariance is mu rho b_k (1 - gamma_k^2) (Monte Carlo over 2^18 nodes);
* a thermal box reaches equipartition: <j_a^2> = rho kT and <drho^2> = rho kT / cs^2
  per node (times 1 - 1/N for the conserved totals), for the projected, BGK and
  MRT operators; these are the variances the fluctuating LBE must produce;
* the extra particle noise of Appendix B has per-step variance kT/(3 pi eta)(1/a - 1/a_L).
"""
import math
import os

import numpy as np
import pytest

from oracle import bruteforce as bf
from oracle import fluct, philox

HERE = os.path.dirname(os.path.abspath(__file__))


def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "philox_kat.txt")) if not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = philox.philox4x32_10(v[0], v[1], v[2], v[3], v[4], v[5])
        assert [int(o) for o in out] == v[6:10]


def test_box_muller_normal_moments():
    n = 1 << 20
    x = philox.philox4x32_10(np.arange(n, dtype=np.uint64), 7, 0, 0, 1234, 5678)
    a, b = philox.box_muller(x[0], x[1])
    z = np.concatenate([a, b])
    assert abs(z.mean()) < 4 / math.sqrt(2 * n)
    assert abs(z.var() - 1) < 4 * math.sqrt(2 / (2 * n))
    assert abs((z ** 4).mean() - 3) < 4 * math.sqrt(96 / (2 * n))
    assert abs(np.corrcoef(a, b)[0, 1]) < 4 / math.sqrt(n)


def test_mode_polynomials_are_w_orthogonal():
    E = fluct.mode_polynomials(bf.C)
    H = np.vstack([np.ones(19), bf.C.T])
    G = (bf.W[None] * E) @ E.T
    assert np.abs(G - np.diag(np.diag(G))).max() < 1e-15
    assert np.all(np.diag(G) > 0.1)
    assert np.abs((bf.W[None] * E) @ H.T).max() < 1e-15
    assert np.linalg.matrix_rank(np.vstack([H, E])) == 19


@pytest.mark.parametrize("rates", [(0.8, None, 2.0), (0.7, 1.5, 0.9), (1.2, None, 1 / 1.2)])
def test_node_noise_conserves_and_has_fdt_covariance(rates):
    tau, tb, lam = rates
    shape = (64, 64, 64)
    kT = 2e-5
    rho = np.full(shape, 1.0) + 1e-3 * np.random.default_rng(0).normal(size=shape)
    z = fluct.lattice_normals(shape, 3, 17, 0x1234_5678_9ABC)
    dn = fluct.lattice_noise(rho, z, kT, tau, tb, lam)
    scale = np.abs(dn).max()            # rounding of 19-term sums of values of this size
    assert np.abs(dn.sum(-1)).max() < 4e-15 * scale
    assert np.abs(dn @ bf.C).max() < 4e-15 * scale
    E = fluct.mode_polynomials(bf.C)
    b = (bf.W[None] * E * E).sum(1)
    m = dn @ E.T / rho[..., None]                      # modes per unit density
    var = (m.reshape(-1, 15) ** 2).mean(0)
    want = kT / fluct.CS2 * b * (1 - fluct.gammas(tau, tb, lam) ** 2)
    assert np.allclose(var, want, rtol=0.02)
    C = np.cov(m.reshape(-1, 15).T)
    off = C - np.diag(np.diag(C))
    assert np.abs(off).max() < 0.02 * want.max()


@pytest.mark.parametrize("op", ["projected", "bgk", "mrt"])
def test_thermal_box_equipartition(op):
    tau = 0.8
    kw = dict(projected=dict(), bgk=dict(ghost_rate=1 / tau), mrt=dict(tau_b=1.4, ghost_rate=0.7))[op]
    shape = (6, 6, 6)
    N = 216
    kT = 1e-5
    box = fluct.FluctBox(shape, tau, kT, seed=99 + len(op), **kw)
    box.step(300)
    jj, rr = [], []
    for t in range(2500):
        box.step(1)
        rho, u = box.moments()
        jj.append(((rho * u) ** 2).mean(axis=(1, 2, 3)))
        rr.append(((rho - 1.0) ** 2).mean())
    jv = np.mean(jj) / (kT * (1 - 1 / N))
    rv = np.mean(rr) / (kT / fluct.CS2 * (1 - 1 / N))
    print("%s: <j^2>/(rho kT) %.3f, <drho^2>/(rho kT/cs2) %.3f" % (op, jv, rv))
    assert abs(jv - 1) < 0.06
    assert abs(rv - 1) < 0.06


def test_particle_noise_variance():
    shape = (8, 8, 8)
    tau, kT = 0.9, 1e-5
    inv_a, inv_aL = 1 / 0.117, 0.77
    n = 4000
    pos = np.random.default_rng(1).uniform(0, 8, (n, 3))
    box = fluct.FluctBox(shape, tau, kT, seed=5, sets=[dict(pos=pos, force=np.zeros((n, 3)), kind="colloid",
                                                            inv_a=inv_a, inv_aL=inv_aL)])
    box.bb.fbar = bf.equilibrium(np.ones(shape), np.zeros(shape + (3,)))
    # the first step interpolates the fluid at rest: the displacement is zeta' alone
    p0 = box.sets[0]["pos"].copy()
    box.step(1)
    d = box.sets[0]["pos"] - p0
    d -= 8 * np.round(d / 8)
    eta = tau / 3
    want = kT / (3 * math.pi * eta) * (inv_a - inv_aL)
    U = box.sets[0]["U"]
    assert np.abs(U).max() == 0.0        # fluid at rest at the first interpolation
    assert abs(d.var() / want - 1) < 4 * math.sqrt(2 / (3 * n))
    assert abs(d.mean()) < 4 * math.sqrt(want / (3 * n))
