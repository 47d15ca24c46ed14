"""Invariants of the whole oracle step (Secs. II-III).

P1 mass: the weights sum to one and propagation is a permutation, so the total
   deviation sum_x drho is unchanged by every step.
P2 momentum: collision adds g, the spread field sums to sum_a F_a, so after n
   steps sum_x jbar = n sum_a F_a and the physical total is (n + 1/2) sum F.
   A uniform body force g0 gives u = (n + 1/2) g0 / rho0 at every node.
P11 multipoles: rotlet and stresslet have zero net force; the first moment
   sum_x x g equals sum_a R_a F_a (so the rotlet torque is 2 d s n and its
   symmetric part vanishes), and the fluid momentum does not change.
P12 linearity at low Mach number: u[F1 + F2] = u[F1] + u[F2] + O(u^2).
"""
import numpy as np
import pytest

import oracle
from oracle import multipole

C_OR, _ = oracle.velocities()
CF = C_OR.astype(float)


def _momentum(df):
    return np.einsum("izyx,ia->a", df, CF)


def test_mass_exactly_conserved():
    rng = np.random.default_rng(1)
    shape = (6, 7, 8)
    box = oracle.Box(shape, 0.8)
    box.df = rng.normal(scale=1e-4, size=(19,) + shape)
    box.sets = [oracle.ForceSet(rng.uniform(0, 6, (3, 3)), rng.normal(scale=1e-4, size=(3, 3)))]
    m0 = box.df.sum()
    for _ in range(30):
        box.step()
    assert abs(box.df.sum() - m0) < 1e-15


@pytest.mark.parametrize("zero_net", [False, True])
def test_momentum_gain_is_n_times_total_force(zero_net):
    rng = np.random.default_rng(2)
    shape = (8, 8, 8)
    F = rng.normal(scale=1e-5, size=(4, 3))
    pos = rng.uniform(0, 8, (4, 3))
    box = oracle.Box(shape, 0.6, zero_net_force=zero_net)
    box.sets = [oracle.ForceSet(pos, F)]
    for n in range(1, 41):
        box.step()
        exp = 0.0 if zero_net else n * F.sum(0)
        assert np.abs(_momentum(box.df) - exp).max() < 1e-18 + 1e-12 * np.abs(F).sum() * n
    rho, u = box.moments()
    phys = (rho[None] * u).sum((1, 2, 3))
    exp = 0.0 if zero_net else 40.5 * F.sum(0)
    assert np.abs(phys - exp).max() < 1e-12 * np.abs(F).sum() * 41


def test_uniform_body_force_velocity():
    """A uniform g0 from spreading a lattice-filling set of equal forces (partition of unity)."""
    shape = (4, 5, 6)
    nz, ny, nx = shape
    g0 = np.array([1e-6, -2e-6, 3e-7])
    # one force per node at the node itself (frac = 0): spreads to exactly g0 everywhere
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    pos = np.stack([x.ravel(), y.ravel(), z.ravel()], 1).astype(float)
    F = np.broadcast_to(g0, pos.shape).copy()
    box = oracle.Box(shape, 0.9)
    box.sets = [oracle.ForceSet(pos, F)]
    assert np.abs(box.force_field() - g0[:, None, None, None]).max() < 1e-20
    for n in range(1, 11):
        box.step()
        rho, u = box.moments()
        assert np.abs(rho - 1.0).max() < 1e-15
        assert np.abs(u - (n + 0.5) * g0[:, None, None, None]).max() < 1e-19


def _random_unit(rng):
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def test_multipole_expansion_moments():
    rng = np.random.default_rng(3)
    for t in (multipole.STRESSLET, multipole.ROTLET):
        ax = _random_unit(rng)
        e1 = rng.normal(size=3)
        e1 -= ax * (ax @ e1)
        e1 /= np.linalg.norm(e1)
        R = np.array([10.3, 11.7, 9.2])
        s, d = 1.3e-5, 2.0
        pos, F = multipole.expand([t], R[None], ax[None], e1[None], [s], d)
        assert np.abs(F.sum(0)).max() < 1e-20
        first = ((pos - R)[:, :, None] * F[:, None, :]).sum(0)     # sum r_a F_b
        sym = 0.5 * (first + first.T)
        anti = 0.5 * (first - first.T)
        if t == multipole.ROTLET:
            assert np.abs(sym).max() < 1e-18
            torque = np.cross(pos - R, F).sum(0)
            assert np.allclose(torque, 2 * d * s * ax, atol=1e-18)
        else:
            assert np.abs(anti).max() < 1e-18
            assert np.allclose(sym, d * s * np.outer(ax, ax), atol=1e-18)


def test_spread_first_moment_of_rotlet_and_fluid_momentum():
    rng = np.random.default_rng(4)
    shape = (16, 16, 16)
    ax = _random_unit(rng)
    e1 = np.cross(ax, [1.0, 0, 0])
    e1 /= np.linalg.norm(e1)
    R = np.array([8.2, 7.6, 8.9])
    pos, F = multipole.expand([multipole.ROTLET], R[None], ax[None], e1[None], [1e-5], 2.0)
    g = oracle.spread(shape, pos, F)
    z, y, x = np.meshgrid(*(np.arange(16.0),) * 3, indexing="ij")
    X = np.stack([x, y, z])
    torque = np.array([(X[(c + 1) % 3] * g[(c + 2) % 3] - X[(c + 2) % 3] * g[(c + 1) % 3]).sum()
                       for c in range(3)])
    assert np.allclose(torque, np.cross(pos, F).sum(0), atol=1e-18)
    assert np.allclose(torque, 2 * 2.0 * 1e-5 * ax, atol=1e-18)
    box = oracle.Box(shape, 0.5)
    box.sets = [oracle.ForceSet(pos, F)]
    box.step(10)
    assert np.abs(_momentum(box.df)).max() < 1e-18


def test_linear_superposition_at_low_mach():
    rng = np.random.default_rng(5)
    shape = (8, 8, 8)
    p1, p2 = rng.uniform(0, 8, (1, 3)), rng.uniform(0, 8, (1, 3))
    F1, F2 = rng.normal(scale=1e-7, size=(1, 3)), rng.normal(scale=1e-7, size=(1, 3))

    def run(sets):
        b = oracle.Box(shape, 0.7)
        b.sets = sets
        b.step(25)
        return b.moments()[1]

    u1 = run([oracle.ForceSet(p1, F1)])
    u2 = run([oracle.ForceSet(p2, F2)])
    u12 = run([oracle.ForceSet(np.vstack([p1, p2]), np.vstack([F1, F2]))])
    scale = np.abs(u12).max()
    assert np.abs(u12 - u1 - u2).max() < 1e-5 * scale


def test_counter_force_keeps_momentum_zero_and_g_mean_zero():
    rng = np.random.default_rng(6)
    shape = (6, 6, 6)
    pos = rng.uniform(0, 6, (5, 3))
    F = np.tile([0.0, 0.0, -1e-6], (5, 1))
    g = oracle.spread(shape, pos, F, zero_net=True)
    assert np.abs(g.sum((1, 2, 3))).max() < 1e-18
