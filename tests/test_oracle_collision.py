"""Pins for the oracle's collision (Eq. fiexp and the A, B that follow it).

* The closed form equals the general scheme Eq. mrtlbe taken literally with an
  explicit collision matrix (oracle/bruteforce.py) whose ghost eigenvalue is
  2/dt ("ghosts projected out") and stress eigenvalue 1/tau.
* The sign printed for the (S - rho v v) term in B cannot be right: with it
  the closed form disagrees with Eq. mrtlbe (the test shows both facts).
* For L = I/tau Eq. mrtlbe reduces to Eq. bgklbe, i.e. textbook BGK with
  Guo forcing at tau_lb = tau + 1/2; at tau = 1/2 the projected-ghost MRT
  relaxes every non-conserved mode fully and equals that BGK step.
* Rest and uniform flow are fixed points; collision conserves mass and adds
  exactly g to the momentum.
"""
import numpy as np
import pytest

import oracle
from oracle import bruteforce as bf

C_OR, W_OR = oracle.velocities()


def _random_node_state(rng, shape, scale=1e-2):
    df = rng.normal(scale=scale, size=(19,) + shape)
    g = rng.normal(scale=scale, size=(3,) + shape)
    return df, g


def _to_brute(df, rho0=1.0):
    fb = np.empty(df.shape[1:] + (19,))
    for i in range(19):
        j = int(np.flatnonzero((C_OR == bf.C[i]).all(1))[0])
        fb[..., i] = bf.W[i] * rho0 + df[j]
    return fb


def _from_brute(fb, rho0=1.0):
    out = np.empty((19,) + fb.shape[:-1])
    for j in range(19):
        i = int(np.flatnonzero((bf.C == C_OR[j]).all(1))[0])
        out[j] = fb[..., i] - bf.W[i] * rho0
    return out


@pytest.mark.parametrize("tau", [0.5, 0.6, 0.8, 1.0, 1.5, 3.0])
def test_closed_form_equals_general_scheme(tau):
    rng = np.random.default_rng(int(tau * 100))
    shape = (4, 4, 4)
    df, g = _random_node_state(rng, shape)
    got, _, _ = oracle.collide(df, g, 1.0, tau)
    ref = _from_brute(bf.collide(_to_brute(df), np.moveaxis(g, 0, -1), tau))
    assert np.abs(got - ref).max() < 1e-15


def test_printed_sign_of_B_disagrees_with_general_scheme():
    """The printed B = S + dt/(tau+dt/2)(S - rho v v + tau(vF + Fv)) is not Eq. mrtlbe."""
    rng = np.random.default_rng(11)
    tau = 0.8
    df, g = _random_node_state(rng, (4, 4, 4))
    fb = _to_brute(df)
    gl = np.moveaxis(g, 0, -1)
    ref = bf.collide(fb, gl, tau)
    rho, v = bf.physical_moments(fb, gl)
    S = np.einsum("...i,iab->...ab", fb, bf.QT)
    vv = np.einsum("...a,...b->...ab", v, v)
    vg = np.einsum("...a,...b->...ab", v, gl)
    A = fb @ bf.C + gl
    om = 1.0 / (tau + 0.5)

    def rebuild(B):
        return bf.W * (rho[..., None] + 3 * A @ bf.C.T
                       + 4.5 * np.einsum("...ab,iab->...i", B, bf.QT))

    printed = S + om * (S - rho[..., None, None] * vv + tau * (vg + np.swapaxes(vg, -1, -2)))
    corrected = S - om * (S - rho[..., None, None] * vv - tau * (vg + np.swapaxes(vg, -1, -2)))
    assert np.abs(rebuild(corrected) - ref).max() < 1e-15
    assert np.abs(rebuild(printed) - ref).max() > 1e-4


@pytest.mark.parametrize("tau", [0.5, 0.7, 1.3])
def test_bgk_special_case_of_general_scheme(tau):
    """Eq. mrtlbe with L = I/tau equals textbook BGK-Guo with tau_lb = tau + 1/2 (Eq. bgklbe)."""
    rng = np.random.default_rng(21)
    df, g = _random_node_state(rng, (3, 3, 3))
    fb = _to_brute(df)
    gl = np.moveaxis(g, 0, -1)
    rho, v = bf.physical_moments(fb, gl)
    f0 = bf.equilibrium(rho, v)
    Phi = bf.forcing(v, gl)
    L = np.eye(19) / tau
    lit = fb + np.linalg.solve(np.eye(19) + 0.5 * L, (-(fb - f0) @ L.T + Phi).reshape(-1, 19).T).T.reshape(fb.shape)
    guo = bf.bgk_guo_collide(fb, gl, tau + 0.5)
    assert np.abs(lit - guo).max() < 1e-15


def test_tau_half_equals_bgk_guo():
    rng = np.random.default_rng(31)
    df, g = _random_node_state(rng, (4, 4, 4))
    got, _, _ = oracle.collide(df, g, 1.0, 0.5)
    guo = _from_brute(bf.bgk_guo_collide(_to_brute(df), np.moveaxis(g, 0, -1), 1.0))
    assert np.abs(got - guo).max() < 1e-15


@pytest.mark.parametrize("tau", [0.5, 0.9])
def test_rest_and_uniform_flow_are_fixed_points(tau):
    shape = (4, 5, 6)
    df0 = np.zeros((19,) + shape)
    s, _, u = oracle.collide(df0, None, 1.0, tau)
    assert np.abs(oracle.stream(s)).max() == 0.0
    rho = np.full(shape, 1.0 + 2e-3)
    u0 = np.array([1e-3, -2e-3, 5e-4])
    uf = np.broadcast_to(u0[:, None, None, None], (3,) + shape).copy()
    df = oracle.equilibrium(rho, uf, 1.0)
    s, r, u = oracle.collide(df, None, 1.0, tau)
    nxt = oracle.stream(s)
    assert np.abs(nxt - df).max() < 1e-13 * np.abs(df).max()
    assert np.abs(u - uf).max() < 1e-13 * np.abs(uf).max()


def test_collision_conserves_mass_and_adds_force():
    rng = np.random.default_rng(41)
    df, g = _random_node_state(rng, (4, 4, 4))
    s, rho, u = oracle.collide(df, g, 1.0, 0.7)
    assert np.abs(s.sum(0) - df.sum(0)).max() < 1e-16
    j0 = np.einsum("i...,ia->a...", df, C_OR.astype(float))
    j1 = np.einsum("i...,ia->a...", s, C_OR.astype(float))
    assert np.abs(j1 - (j0 + g)).max() < 1e-16
    # physical velocity of Eq. macrovariables2
    assert np.abs(u * rho - (j0 + 0.5 * g)).max() < 1e-16


def test_post_collision_has_no_ghosts_and_relaxed_stress():
    """Post-collision ghost moments vanish; stress = Sbar - omega(Sbar - rho uu - tau(ug+gu))."""
    rng = np.random.default_rng(51)
    tau = 1.2
    df, g = _random_node_state(rng, (3, 3, 3))
    s, rho, u = oracle.collide(df, g, 1.0, tau)
    M = bf.moment_matrix()
    fb = _to_brute(s)
    ghosts = fb @ M[10:].T
    assert np.abs(ghosts).max() < 1e-14
    S0 = np.einsum("...i,iab->...ab", _to_brute(df), bf.QT)
    S1 = np.einsum("...i,iab->...ab", fb, bf.QT)
    ul = np.moveaxis(u, 0, -1)
    gl = np.moveaxis(g, 0, -1)
    uu = np.einsum("...a,...b->...ab", ul, ul) * rho[..., None, None]
    ug = np.einsum("...a,...b->...ab", ul, gl)
    om = 1 / (tau + 0.5)
    exp = S0 - om * (S0 - uu - tau * (ug + np.swapaxes(ug, -1, -2)))
    assert np.abs(S1 - exp).max() < 1e-15
