"""Pins for the general forced MRT oracle (Eq. mrtlbe with separate shear,
bulk and ghost rates) against closed forms.

The brute-force oracle builds L = M^-1 diag(lambda) M; these tests tie it to
facts that do not go through that construction:

* with lambda_g = 1/tau and tau_b = tau it is the textbook BGK step with
  Guo forcing (Eq. bgklbe, tau_lb = tau + 1/2);
* with lambda_g = 2 and tau_b = tau it is the projected operator of
  Eq. fiexp (the C oracle);
* a ghost perturbation w_i psi(c_i), with psi a polynomial written here and
  w-orthogonal to 1, c, Q, is multiplied by (1 - lambda_g/2)/(1 + lambda_g/2);
  a bulk perturbation w_i (c_i^2 - 1) by 1 - 1/(tau_b + 1/2); a shear
  perturbation w_i c_ix c_iy by 1 - 1/(tau + 1/2);
* mass is kept and momentum gains g (A of Eq. fiexp) for any rates.
"""
import numpy as np
import pytest

import oracle
from oracle import bruteforce as bf


def _node_state(rng, shape):
    df = rng.normal(scale=1e-3, size=(19,) + shape)
    g = rng.normal(scale=1e-4, size=(3,) + shape)
    return df, g


def _to_brute(df):
    bb = bf.BruteBox(df.shape[1:], 1.0, 1.0)
    bb.set_deviation_from(df, oracle.velocities()[0])
    return bb.fbar


def _rest(rho=1.0):
    return bf.equilibrium(np.array(rho), np.zeros(3))


@pytest.mark.parametrize("tau", [0.5, 0.8, 1.7])
def test_bgk_rates_equal_textbook_bgk_guo(tau):
    rng = np.random.default_rng(5)
    df, g = _node_state(rng, (3, 3, 2))
    fb = _to_brute(df)
    gl = np.moveaxis(g, 0, -1)
    got = bf.collide(fb, gl, tau, tau, 1.0 / tau)
    ref = bf.bgk_guo_collide(fb, gl, tau + 0.5)
    assert np.abs(got - ref).max() < 2e-15


@pytest.mark.parametrize("tau", [0.5, 1.1])
def test_default_rates_equal_projected_c_oracle(tau):
    rng = np.random.default_rng(6)
    df, g = _node_state(rng, (3, 2, 4))
    fb = _to_brute(df)
    got = bf.collide(fb, np.moveaxis(g, 0, -1), tau, tau, 2.0)
    ref, _, _ = oracle.collide(df, g, 1.0, tau)
    bb = bf.BruteBox(df.shape[1:], tau, 1.0)
    bb.fbar = got
    assert np.abs(bb.deviation_in(oracle.velocities()[0]) - ref).max() < 2e-15


@pytest.mark.parametrize("lam", [0.3, 1.0, 1.7, 2.0, 2.5])
@pytest.mark.parametrize("ghost", ["cx(cy2-cz2)", "3c4-6c2+1", "cz(cx2-cy2)"])
def test_ghost_perturbation_decays_by_kappa(lam, ghost):
    c = bf.C
    c2 = (c * c).sum(1)
    psi = {"cx(cy2-cz2)": c[:, 0] * (c[:, 1] ** 2 - c[:, 2] ** 2),
           "3c4-6c2+1": 3 * c2 ** 2 - 6 * c2 + 1,
           "cz(cx2-cy2)": c[:, 2] * (c[:, 0] ** 2 - c[:, 1] ** 2)}[ghost]
    f0 = _rest(1.0 + 3e-3)
    eps = 1e-3
    fb = f0 + eps * bf.W * psi
    out = bf.collide(fb[None], np.zeros((1, 3)), 0.9, 1.3, lam)[0]
    kappa = (1 - lam / 2) / (1 + lam / 2)
    assert np.abs(out - (f0 + kappa * eps * bf.W * psi)).max() < 1e-16


@pytest.mark.parametrize("tau_b", [0.5, 0.9, 3.0])
def test_bulk_perturbation_relaxes_with_tau_bulk(tau_b):
    c2 = (bf.C * bf.C).sum(1)
    f0 = _rest(1.0)
    eps = 2e-3
    fb = f0 + eps * bf.W * (c2 - 1)
    out = bf.collide(fb[None], np.zeros((1, 3)), 0.7, tau_b, 1.2)[0]
    assert np.abs(out - (f0 + (1 - 1 / (tau_b + 0.5)) * eps * bf.W * (c2 - 1))).max() < 1e-16


@pytest.mark.parametrize("tau", [0.55, 1.4])
def test_shear_perturbation_relaxes_with_tau(tau):
    f0 = _rest(1.0)
    eps = 2e-3
    shear = bf.C[:, 0] * bf.C[:, 1]
    fb = f0 + eps * bf.W * shear
    out = bf.collide(fb[None], np.zeros((1, 3)), tau, 2.5, 0.4)[0]
    assert np.abs(out - (f0 + (1 - 1 / (tau + 0.5)) * eps * bf.W * shear)).max() < 1e-16


@pytest.mark.parametrize("rates", [(0.6, 0.6, 2.0), (0.8, 2.0, 0.5), (1.5, 0.7, 1.9)])
def test_mass_kept_momentum_gains_force(rates):
    tau, tb, lam = rates
    rng = np.random.default_rng(8)
    df, g = _node_state(rng, (2, 3, 3))
    fb = _to_brute(df)
    gl = np.moveaxis(g, 0, -1)
    out = bf.collide(fb, gl, tau, tb, lam)
    assert np.abs(out.sum(-1) - fb.sum(-1)).max() < 1e-15
    assert np.abs(out @ bf.C - (fb @ bf.C + gl)).max() < 2e-16   # rounding of sums of 19 terms ~ 0.05


@pytest.mark.parametrize("rates", [(0.6, 1.9), (1.2, 0.55)])
def test_projected_ghosts_with_bulk_rate_match_moment_form(rates):
    """lambda_g = 2: the post-collision state is w_i [rho + 3 A.c + 9/2 B:Q] with B's traceless
    part relaxed at 1/(tau + 1/2) and its trace at 1/(tau_b + 1/2) (both driven as in Eq. fiexp)."""
    tau, tb = rates
    rng = np.random.default_rng(9)
    df, g = _node_state(rng, (2, 2, 3))
    fb = _to_brute(df)
    gl = np.moveaxis(g, 0, -1)
    out = bf.collide(fb, gl, tau, tb, 2.0)
    rho, v = bf.physical_moments(fb, gl)
    S = np.einsum("...i,iab->...ab", fb, bf.QT)
    A = fb @ bf.C + gl
    vv = np.einsum("...a,...b->...ab", v, v)
    vg = np.einsum("...a,...b->...ab", v, gl)
    vg = vg + np.swapaxes(vg, -1, -2)
    I = np.eye(3)

    def dev(X):
        return X - np.trace(X, axis1=-2, axis2=-1)[..., None, None] * I / 3

    def tr(X):
        return np.trace(X, axis1=-2, axis2=-1)[..., None, None] * I / 3

    om, omb = 1 / (tau + 0.5), 1 / (tb + 0.5)
    B = S - om * dev(S - rho[..., None, None] * vv - tau * vg) - omb * tr(S - rho[..., None, None] * vv - tb * vg)
    ref = bf.W * (rho[..., None] + 3 * A @ bf.C.T + 4.5 * np.einsum("...ab,iab->...i", B, bf.QT))
    assert np.abs(out - ref).max() < 2e-15
