"""Singular forces on curves and surfaces (Sec. I; Eq. singularF with a line or
area measure), discretised on markers.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper names polymers (curves) and interfaces (surfaces) as singular force
densities F(r) = int f(R(l)) delta(r - R(l)) dl and leaves their models open.
Reading taken here: the manifold is carried by markers; the integral becomes a
sum of marker forces (the measure dl absorbed in each marker's force), spread
and interpolated with the same Peskin kernel as point forces, and the markers
move with the interpolated fluid velocity (R <- R + U, no point-particle
mobility correction).

* Chain (polymer as a curve): markers 0..n-1 grouped in chains of m
  consecutive markers; each pair (i, i+1) in one chain is a Hookean spring of
  stiffness k and rest length l0, the force on i being
  k (|d| - l0) d / |d|, d = R_{i+1} - R_i (minimum image), and its opposite on
  i+1; plus an optional external force per marker.
* Surface (interface): a closed triangulated surface of tension gamma, energy
  gamma * area; vertex force -gamma dA/dR_v, where for a triangle (a, b, c)
  ordered counter-clockwise about its unit normal n, dA/da = n x (c - b) / 2.
"""
from __future__ import annotations

import numpy as np

from . import advect, collide, interp, moments, spread, stream


def _min_image(d, L):
    return d - L * np.round(d / L)


def chain_forces(pos, chain_len, k, l0, L, ext=None):
    """Spring forces of chains of chain_len consecutive markers; L = (nx, ny, nz)."""
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    n = len(pos)
    F = np.zeros((n, 3)) if ext is None else np.array(ext, dtype=np.float64).reshape(n, 3).copy()
    i = np.arange(n - 1)
    i = i[(i + 1) % chain_len != 0]                      # springs (i, i + 1) inside a chain
    d = _min_image(pos[i + 1] - pos[i], np.asarray(L, dtype=np.float64))
    r = np.sqrt((d * d).sum(1))
    f = (k * (r - l0) / r)[:, None] * d
    np.add.at(F, i, f)
    np.add.at(F, i + 1, -f)
    return F


def triangle_area_gradients(pos, tri, L):
    """[ntri, 3, 3]: per triangle the gradients dA/dR of its area for vertices a, b, c."""
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    tri = np.asarray(tri).reshape(-1, 3)
    Lv = np.asarray(L, dtype=np.float64)
    pa = pos[tri[:, 0]]
    pb = pa + _min_image(pos[tri[:, 1]] - pa, Lv)
    pc = pa + _min_image(pos[tri[:, 2]] - pa, Lv)
    cr = np.cross(pb - pa, pc - pa)
    n = cr / np.sqrt((cr * cr).sum(1))[:, None]
    return 0.5 * np.stack([np.cross(n, pc - pb), np.cross(n, pa - pc), np.cross(n, pb - pa)], 1)


def surface_forces(pos, tri, tension, L, ext=None):
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    tri = np.asarray(tri).reshape(-1, 3)
    F = np.zeros_like(pos) if ext is None else np.array(ext, dtype=np.float64).reshape(pos.shape).copy()
    G = triangle_area_gradients(pos, tri, L)
    for j in range(3):
        np.add.at(F, tri[:, j], -tension * G[:, j])
    return F


def surface_area(pos, tri, L):
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    tri = np.asarray(tri).reshape(-1, 3)
    Lv = np.asarray(L, dtype=np.float64)
    pb = _min_image(pos[tri[:, 1]] - pos[tri[:, 0]], Lv)
    pc = _min_image(pos[tri[:, 2]] - pos[tri[:, 0]], Lv)
    return float(0.5 * np.sqrt((np.cross(pb, pc) ** 2).sum(1)).sum())


def icosphere(center, radius, levels):
    """Triangulated sphere: an icosahedron subdivided `levels` times, projected to the sphere,
    triangles counter-clockwise seen from outside."""
    t = (1 + 5 ** 0.5) / 2
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6),
         (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10),
         (8, 6, 7), (9, 8, 1)]
    verts = [np.array(p, dtype=np.float64) / np.linalg.norm(p) for p in v]
    for _ in range(levels):
        cache = {}

        def mid(i, j):
            key = (min(i, j), max(i, j))
            if key not in cache:
                m = verts[i] + verts[j]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        f = nf
    V = np.array(verts) * radius + np.asarray(center, dtype=np.float64)
    F = np.array(f, dtype=np.int32)
    # orient counter-clockwise about the outward normal
    for k, (a, b, c) in enumerate(F):
        n = np.cross(V[b] - V[a], V[c] - V[a])
        if np.dot(n, (V[a] + V[b] + V[c]) / 3 - center) < 0:
            F[k] = (a, c, b)
    return V, F


class ElasticBox:
    """One periodic box stepped by the C oracle (projected operator) with marker sets whose
    forces are recomputed from their configuration every step and which move with the fluid.
    sets: dicts with pos and either kind='chain' (chain_len, k, l0) or kind='surface' (tri,
    tension); optional ext (external force per marker)."""

    def __init__(self, shape, tau, rho0=1.0, zero_net=False, sets=()):
        self.shape = tuple(shape)
        self.tau, self.rho0, self.zero_net = tau, rho0, zero_net
        self.df = np.zeros((19,) + self.shape)
        self.sets = [dict(s, pos=np.array(s["pos"], dtype=np.float64).reshape(-1, 3)) for s in sets]
        self.L = (self.shape[2], self.shape[1], self.shape[0])

    def forces(self, s):
        if s["kind"] == "chain":
            return chain_forces(s["pos"], s["chain_len"], s["k"], s["l0"], self.L, s.get("ext"))
        return surface_forces(s["pos"], s["tri"], s["tension"], self.L, s.get("ext"))

    def _field(self):
        for s in self.sets:
            s["F"] = self.forces(s)
        pos = np.concatenate([s["pos"] for s in self.sets])
        frc = np.concatenate([s["F"] for s in self.sets])
        return spread(self.shape, pos, frc, self.zero_net)

    def step(self, n=1):
        for _ in range(n):
            g = self._field()
            dfs, rho, u = collide(self.df, g, self.rho0, self.tau)
            for s in self.sets:
                s["U"] = interp(u, s["pos"])
            self.df = stream(dfs)
            for s in self.sets:     # markers move with the fluid: the Sec. IV update without mobility terms
                s["pos"] = advect(self.shape, self.rho0, self.tau, s["pos"], s["F"], s["U"], 0.0, 0.0)

    def moments(self):
        return moments(self.df, self._field(), self.rho0)
