"""Fluctuating forced LB with Brownian point colloids (Sec. II, Sec. IV,
Appendix B).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper takes the fluctuating LB equation from its reference on discrete
kinetic fluctuations (Adhikari et al. 2005) and states only what it must
achieve (thermodynamically correct variances of the local mass and momentum
densities) and the extra particle noise.  Reading taken here:

* After the deterministic collision of Eq. mrtlbe (brute force, any shear,
  bulk and ghost rates), each non-conserved mode k of the post-collision
  auxiliary populations receives a random increment phi_k with variance
  mu rho b_k (1 - gamma_k^2): mu = kT / cs^2, rho the node's density,
  b_k = sum_i w_i e_k(c_i)^2 the mode's norm, gamma_k the factor the collision
  applies to the mode's non-equilibrium part (1 - 1/(tau_b + 1/2) bulk,
  1 - 1/(tau + 1/2) shear, (1 - r/2)/(1 + r/2) ghosts at rate r).  Mass and
  momentum receive none.  In population space the increment is
  w_i sum_k e_k(c_i) phi_k / b_k.
* Modes: the fifteen non-conserved D3Q19 polynomials of the orthogonal basis
  published by Duenweg, Schiller and Ladd (Phys. Rev. E 76, 036704, 2007):
  bulk c^2 - 1; shear 3 c_x^2 - c^2, c_y^2 - c_z^2, c_x c_y, c_x c_z,
  c_y c_z; ghosts (3 c^2 - 5) c_a (three), (c_y^2 - c_z^2) c_x,
  (c_z^2 - c_x^2) c_y, (c_x^2 - c_y^2) c_z, 3 c^4 - 6 c^2 + 1,
  (2 c^2 - 3)(3 c_x^2 - c^2), (2 c^2 - 3)(c_y^2 - c_z^2).  They are mutually
  w-orthogonal and w-orthogonal to 1 and c.
* Random numbers: Philox4x32-10, key (seed low 32 bits, seed high 32 bits).
  Node noise of step t (t = steps taken before it) for node n = (z ny + y) nx + x
  of box b: counter (n, b, t mod 2^32, (t >> 32) << 4 | j), j = 0..3, the
  sixteen normals (Box-Muller on consecutive pairs) feeding modes 0..14 in
  the order above.  Particle noise: counter (p, 2^32 - 1, t mod 2^32,
  (t >> 32) << 4), p the particle's index over the context's sets in
  registration order; normals 0..2 feed x, y, z.
* Particle (Appendix B): each step R <- R + U + F/(6 pi eta)(1/a - 1/a_L)
  + sqrt(kT/(3 pi eta) (1/a - 1/a_L)) N, eta = rho0 tau / 3, the noise term
  being the extra zeta' whose variance the fluctuation-dissipation theorem
  fixes.
"""
from __future__ import annotations

import math

import numpy as np

from . import advect, interp, spread
from . import bruteforce as bf
from . import philox

CS2 = 1.0 / 3.0
NMODES = 15
PARTICLE_STREAM = 0xFFFFFFFF


def mode_polynomials(c):
    """The fifteen non-conserved mode polynomials evaluated on velocities c [q, 3] -> [15, q]."""
    cx, cy, cz = (np.asarray(c, dtype=np.float64)[:, a] for a in range(3))
    c2 = cx * cx + cy * cy + cz * cz
    return np.array([
        c2 - 1, 3 * cx * cx - c2, cy * cy - cz * cz, cx * cy, cx * cz, cy * cz,
        (3 * c2 - 5) * cx, (3 * c2 - 5) * cy, (3 * c2 - 5) * cz,
        (cy * cy - cz * cz) * cx, (cz * cz - cx * cx) * cy, (cx * cx - cy * cy) * cz,
        3 * c2 * c2 - 6 * c2 + 1, (2 * c2 - 3) * (3 * cx * cx - c2), (2 * c2 - 3) * (cy * cy - cz * cz)])


def gammas(tau, tau_b=None, ghost_rate=2.0):
    tb = tau if tau_b is None else tau_b
    return np.array([1 - 1 / (tb + 0.5)] + [1 - 1 / (tau + 0.5)] * 5 + [(1 - ghost_rate / 2) / (1 + ghost_rate / 2)] * 9)


def lattice_normals(shape, box, t, seed):
    """[nz, ny, nx, 15] standard normals of the node noise of step t."""
    nz, ny, nx = shape
    n = np.arange(nz * ny * nx, dtype=np.uint64)
    z = philox.normals(n, box, t & 0xFFFFFFFF, ((t >> 32) & 0x0FFFFFFF) << 4, 4, seed & 0xFFFFFFFF,
                       (seed >> 32) & 0xFFFFFFFF)
    return np.stack(z[:NMODES], -1).reshape(tuple(shape) + (NMODES,))


def lattice_noise(rho, normals, kT, tau, tau_b=None, ghost_rate=2.0):
    """Population-space increment [.., 19] (brute-force velocity order) for node densities rho [..]."""
    E = mode_polynomials(bf.C)                  # [15, 19]
    b = (bf.W[None] * E * E).sum(1)             # norms
    mu = kT / CS2
    amp = np.sqrt(mu * rho[..., None] * (1 - gammas(tau, tau_b, ghost_rate) ** 2) / b)
    return bf.W * ((amp * normals) @ E)


def particle_normals(npts, t, seed):
    z = philox.normals(np.arange(npts, dtype=np.uint64), PARTICLE_STREAM, t & 0xFFFFFFFF,
                       ((t >> 32) & 0x0FFFFFFF) << 4, 1, seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    return np.stack(z[:3], -1)


class FluctBox:
    """One periodic box: brute-force collision (Eq. mrtlbe) + thermal noise + propagation;
    point sets spread and interpolated with the C oracle, colloids advanced with the extra
    Brownian displacement.  sets: list of dicts pos, force, kind ('static' | 'colloid'),
    inv_a, inv_aL."""

    def __init__(self, shape, tau, kT, seed, rho0=1.0, tau_b=None, ghost_rate=2.0, box=0, zero_net=False, sets=()):
        self.shape = tuple(shape)
        self.tau, self.tau_b, self.ghost_rate = tau, tau_b, ghost_rate
        self.kT, self.seed, self.rho0, self.box = kT, seed, rho0, box
        self.zero_net = zero_net
        self.bb = bf.BruteBox(self.shape, tau, rho0, tau_b, ghost_rate)
        self.sets = [dict(s, pos=np.array(s["pos"], dtype=np.float64).reshape(-1, 3),
                          force=np.array(s["force"], dtype=np.float64).reshape(-1, 3)) for s in sets]
        self.t = 0

    def _g(self):
        if not self.sets:
            return np.zeros(self.shape + (3,))
        pos = np.concatenate([s["pos"] for s in self.sets])
        frc = np.concatenate([s["force"] for s in self.sets])
        return np.moveaxis(spread(self.shape, pos, frc, self.zero_net), 0, -1)

    def step(self, n=1):
        eta = self.rho0 * self.tau * CS2
        for _ in range(n):
            g = self._g()
            rho, v = self.bb.moments(g)
            u = np.ascontiguousarray(np.moveaxis(v, -1, 0))
            for s in self.sets:
                s["U"] = interp(u, s["pos"])
            post = bf.collide(self.bb.fbar, g, self.tau, self.tau_b, self.ghost_rate)
            if self.kT > 0:
                post = post + lattice_noise(rho, lattice_normals(self.shape, self.box, self.t, self.seed), self.kT,
                                            self.tau, self.tau_b, self.ghost_rate)
            self.bb.fbar = bf.stream(post)
            off = 0
            for s in self.sets:
                m = len(s["pos"])
                if s["kind"] == "colloid":
                    U = s["U"]
                    if self.kT > 0:
                        d = np.broadcast_to(np.asarray(s["inv_a"]) - np.asarray(s["inv_aL"]), (m,))
                        amp = np.sqrt(self.kT / (3 * math.pi * eta) * d)
                        U = U + amp[..., None] * particle_normals(off + m, self.t, self.seed)[off:]
                    s["pos"] = advect(self.shape, self.rho0, self.tau, s["pos"], s["force"], U, s["inv_a"], s["inv_aL"])
                off += m
            self.t += 1

    def moments(self):
        """Physical (rho [..], u [3, ..]) with the current forces."""
        rho, v = self.bb.moments(self._g())
        return rho, np.moveaxis(v, -1, 0)
