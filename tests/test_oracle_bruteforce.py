"""Brute force on tiny grids: the oracle's whole step equals Eq. mrtlbe taken
literally (explicit collision matrix, full populations, np.roll streaming,
dense minimum-image spreading) over 20 steps, with random initial states and
one to three random point forces.  The brute force carries full populations
of size ~w_i rho0, so the bound is absolute at a few ulp of rho0 = 1 per step
(2e-15), far below any missing term (the state is ~3e-4, u ~ 1e-3)."""
import numpy as np
import pytest

import oracle
from oracle import bruteforce as bf

C_OR, _ = oracle.velocities()


@pytest.mark.parametrize("shape,nf,zero_net,tau", [
    ((4, 4, 4), 1, False, 0.5),
    ((5, 5, 5), 2, False, 0.8),
    ((6, 6, 6), 3, True, 1.1),
    ((4, 5, 6), 3, False, 0.65),
    ((6, 4, 5), 2, True, 0.5),
])
def test_oracle_equals_literal_scheme(shape, nf, zero_net, tau):
    rng = np.random.default_rng(sum(shape) * 7 + nf)
    nz, ny, nx = shape
    df = rng.normal(scale=1e-3, size=(19,) + shape)
    pos = rng.uniform(0, 1, size=(nf, 3)) * np.array([nx, ny, nz])
    F = rng.normal(scale=1e-3, size=(nf, 3))
    box = oracle.Box(shape, tau, 1.0, zero_net_force=zero_net)
    box.df = df.copy()
    box.sets = [oracle.ForceSet(pos, F)]
    bb = bf.BruteBox(shape, tau, 1.0)
    bb.set_deviation_from(df, C_OR)
    gd = bf.spread_dense(shape, pos, F, zero_net)
    for _ in range(20):
        box.step()
        bb.step(gd)
    ref = bb.deviation_in(C_OR)
    assert np.abs(box.df - ref).max() <= 2e-15
    # physical moments through both
    rho_o, u_o = box.moments()
    rho_b, u_b = bb.moments(gd)
    assert np.abs(rho_o - rho_b).max() < 1e-14
    assert np.abs(u_o - np.moveaxis(u_b, -1, 0)).max() <= 2e-15
    # interpolation at the forces
    U = box.interp_velocity(pos)
    Ub = bf.interp_dense(u_b, pos)
    assert np.abs(U - Ub).max() <= 2e-15
