"""Brute-force form of the general forced MRT scheme, Eq. mrtlbe (Sec. II).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Works on full auxiliary populations fbar (not deviations) and builds the
collision matrix L explicitly:  L = M^-1 diag(lambda) M, where the rows of M
are the moments 1, c, the trace of Q (bulk), five traceless combinations of
Q (shear) and nine ghost moments chosen orthogonal to them in the w-weighted
inner product.  Eigenvalues: 0 on mass and momentum (the conservation
constraints of Eq. conservation), 1/tau on the shear moments, 1/tau_b on the
bulk moment (tau_b = tau unless given), and lambda_g on the ghosts.  The
paper's operator of Eq. fiexp is tau_b = tau, lambda_g = 2/dt (then
(1 + L/2)^-1 L is the identity on the ghosts: they are projected out); the
single-relaxation-time operator of Eq. bgklbe is tau_b = tau,
lambda_g = 1/tau.  With one rate for all nine ghosts the operator does not
depend on how the ghost subspace is spanned.  One step is taken literally as

    fbar(x + c_i, t + 1) = fbar(x, t) + (1 + L/2)^-1 [ -L (fbar - f0) + Phi ]

with f0 from Eq. eqf at the physical (rho, v) of Eq. macrovariables2 and
Phi_i = w_i [ g.c_i / cs^2 + (v g + g v):Q_i / (2 cs^4) ]  (g = rho F),
the linear solve done by numpy.  The velocity table here is written
independently of the C oracle's, in a different order.
"""
from __future__ import annotations

import itertools

import numpy as np

CS2 = 1.0 / 3.0


def d3q19():
    """D3Q19 listed as rest, edges, faces (a different order from the C oracle)."""
    vel = [(0, 0, 0)]
    for v in itertools.product((-1, 0, 1), repeat=3):
        if sum(abs(t) for t in v) == 2:
            vel.append(v)
    for v in itertools.product((-1, 0, 1), repeat=3):
        if sum(abs(t) for t in v) == 1:
            vel.append(v)
    c = np.array(vel, dtype=np.float64)
    n2 = (c * c).sum(1)
    w = np.where(n2 == 0, 1.0 / 3.0, np.where(n2 == 1, 1.0 / 18.0, 1.0 / 36.0))
    return c, w


C, W = d3q19()
I3 = np.eye(3)
QT = np.einsum("ia,ib->iab", C, C) - CS2 * I3[None]  # Q_i tensor [19, 3, 3]


def moment_matrix():
    """Rows: 1, c_x, c_y, c_z, the bulk moment tr Q, five traceless stress moments
    (Q_xx - Q_yy, Q_xx + Q_yy - 2 Q_zz, Q_xy, Q_xz, Q_yz), nine w-orthogonal ghosts."""
    rows = [np.ones(19), C[:, 0], C[:, 1], C[:, 2], QT[:, 0, 0] + QT[:, 1, 1] + QT[:, 2, 2],
            QT[:, 0, 0] - QT[:, 1, 1], QT[:, 0, 0] + QT[:, 1, 1] - 2 * QT[:, 2, 2],
            QT[:, 0, 1], QT[:, 0, 2], QT[:, 1, 2]]
    H = np.array(rows)                           # [10, 19]
    sw = np.sqrt(W)
    # orthogonal complement of span(sqrt(w) * h) in R^19, mapped back by 1/sqrt(w)
    U, s, Vt = np.linalg.svd((H * sw[None]).T, full_matrices=True)
    comp = U[:, 10:].T                           # [9, 19], orthonormal, orthogonal to sqrt(w) h
    ghosts = comp / sw[None]
    return np.vstack([H, ghosts])


def collision_matrix(tau: float, tau_bulk: float | None = None, ghost_rate: float = 2.0) -> np.ndarray:
    M = moment_matrix()
    tb = tau if tau_bulk is None else tau_bulk
    lam = np.array([0.0] * 4 + [1.0 / tb] + [1.0 / tau] * 5 + [ghost_rate] * 9)
    return np.linalg.solve(M, np.diag(lam) @ M)


def equilibrium(rho, v):
    """Eq. eqf, per node: rho [..], v [.., 3] -> f0 [.., 19]."""
    vc = v @ C.T
    vvQ = np.einsum("...a,...b,iab->...i", v, v, QT)
    return W * (rho[..., None] + rho[..., None] * vc / CS2 + rho[..., None] * vvQ / (2 * CS2 ** 2))


def forcing(v, g):
    """Phi_i = w_i [ g.c_i / cs^2 + (v g + g v):Q_i / (2 cs^4) ]."""
    gc = g @ C.T
    vgQ = np.einsum("...a,...b,iab->...i", v, g, QT) + np.einsum("...a,...b,iab->...i", g, v, QT)
    return W * (gc / CS2 + vgQ / (2 * CS2 ** 2))


def physical_moments(fbar, g):
    """Eq. macrovariables2: rho = sum fbar, rho v = sum fbar c + g/2."""
    rho = fbar.sum(-1)
    v = (fbar @ C + 0.5 * g) / rho[..., None]
    return rho, v


def collide(fbar, g, tau, tau_bulk=None, ghost_rate=2.0):
    """Post-collision fbar* for every node; fbar [.., 19], g [.., 3]."""
    L = collision_matrix(tau, tau_bulk, ghost_rate)
    rho, v = physical_moments(fbar, g)
    f0 = equilibrium(rho, v)
    Phi = forcing(v, g)
    rhs = -(fbar - f0) @ L.T + Phi
    R = np.linalg.solve(np.eye(19) + 0.5 * L, rhs.reshape(-1, 19).T).T.reshape(rhs.shape)
    return fbar + R


def stream(fbar):
    """fbar_i(x + c_i) = fbar*_i(x); fbar [nz, ny, nx, 19]."""
    out = np.empty_like(fbar)
    for i in range(19):
        cx, cy, cz = (int(t) for t in C[i])
        out[..., i] = np.roll(fbar[..., i], shift=(cz, cy, cx), axis=(0, 1, 2))
    return out


def bgk_guo_collide(fbar, g, tau_lb):
    """Textbook BGK with Guo's forcing (single relaxation time tau_lb):
       fbar* = fbar - (fbar - f0)/tau_lb + (1 - 1/(2 tau_lb)) w_i [3 (c_i - u).g + 9 (c_i.u)(c_i.g)]."""
    rho, u = physical_moments(fbar, g)
    f0 = equilibrium(rho, u)
    cu = u @ C.T
    cg = g @ C.T
    ug = (u * g).sum(-1, keepdims=True)
    Fi = W * (3.0 * (cg - ug) + 9.0 * cu * cg)
    return fbar - (fbar - f0) / tau_lb + (1.0 - 0.5 / tau_lb) * Fi


def peskin_1d(r):
    """Eq. deltadef, vectorised, written independently of the C oracle."""
    a = np.abs(np.asarray(r, dtype=np.float64))
    inner = (3 - 2 * a + np.sqrt(np.clip(1 + 4 * a - 4 * a * a, 0, None))) / 8
    outer = (5 - 2 * a - np.sqrt(np.clip(-7 + 12 * a - 4 * a * a, 0, None))) / 8
    return np.where(a <= 1, inner, np.where(a <= 2, outer, 0.0))


def spread_dense(shape, pos, force, zero_net=False):
    """g(x) = sum_a F_a deltaP(x - R_a) by brute force over every node and particle,
    using the minimum-image distance; returns [nz, ny, nx, 3]."""
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    g = np.zeros((nz, ny, nx, 3))
    for R, F in zip(np.reshape(pos, (-1, 3)), np.reshape(force, (-1, 3))):
        d = []
        for coord, Rc, L in ((x, R[0], nx), (y, R[1], ny), (z, R[2], nz)):
            dd = coord - Rc
            dd = dd - L * np.round(dd / L)
            d.append(dd)
        wgt = peskin_1d(d[0]) * peskin_1d(d[1]) * peskin_1d(d[2])
        g += wgt[..., None] * np.asarray(F)[None, None, None, :]
    if zero_net and len(np.reshape(pos, (-1, 3))):
        g -= np.reshape(force, (-1, 3)).sum(0) / (nx * ny * nz)
    return g


def interp_dense(u, pos):
    """U(R) = sum_x u(x) deltaP(x - R), brute force; u [nz, ny, nx, 3]."""
    nz, ny, nx, _ = u.shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    out = []
    for R in np.reshape(pos, (-1, 3)):
        d = []
        for coord, Rc, L in ((x, R[0], nx), (y, R[1], ny), (z, R[2], nz)):
            dd = coord - Rc
            dd = dd - L * np.round(dd / L)
            d.append(dd)
        wgt = peskin_1d(d[0]) * peskin_1d(d[1]) * peskin_1d(d[2])
        out.append((wgt[..., None] * u).sum((0, 1, 2)))
    return np.array(out).reshape(-1, 3)


class BruteBox:
    """Tiny periodic box stepped with the literal Eq. mrtlbe."""

    def __init__(self, shape, tau, rho0=1.0, tau_bulk=None, ghost_rate=2.0):
        self.shape = tuple(shape)
        self.tau = tau
        self.tau_bulk = tau_bulk
        self.ghost_rate = ghost_rate
        self.rho0 = rho0
        self.fbar = np.broadcast_to(W * rho0, self.shape + (19,)).copy()

    def set_deviation_from(self, df_c_order, c_table):
        """Load a state given as deviations in another velocity order ([19, nz, ny, nx])."""
        for i in range(19):
            j = int(np.flatnonzero((c_table == C[i]).all(1))[0])
            self.fbar[..., i] = W[i] * self.rho0 + df_c_order[j]

    def deviation_in(self, c_table):
        out = np.empty((19,) + self.shape)
        for j in range(19):
            i = int(np.flatnonzero((C == c_table[j]).all(1))[0])
            out[j] = self.fbar[..., i] - W[i] * self.rho0
        return out

    def step(self, g):
        self.fbar = stream(collide(self.fbar, g, self.tau, self.tau_bulk, self.ghost_rate))

    def moments(self, g):
        return physical_moments(self.fbar, g)
