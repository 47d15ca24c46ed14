"""Seeded synthetic inputs shaped like the paper's workloads.

Only random draws live here (positions, orientations, strengths, box
parameters); none of the method's arithmetic.  Both the HIP path and the
oracle receive exactly these arrays.  Seeds are 20261200 + workload index.

  stokeslet_box    one point force F = (0, 0, 1e-5) at a uniform position
                   in a 32^3 box (the Fig. 1 validation problem)
  singularities    64 Stokeslets / stresslets / rotlets, type uniform,
                   strength s ~ U[-1e-5, 1e-5], axis uniform on the sphere,
                   second axis uniform in the normal plane, centres uniform,
                   separation 2 (Figs. 2-3 multipoles)
  colloids         n equal gravity forces (0, 0, -1e-6) at uniform positions
                   (the sedimenting suspensions of Sec. IV, Table 1)
  mobility_boxes   per box 1..8 fixed colloids at the first k sites of the
                   2x2x2 sub-lattice of spacing L/2, sub-node offsets
                   U[0, 1)^3, tau_b ~ U[0.6, 1.5]
  droplets         n spherical interfaces (geodesic triangulations of the
                   icosahedron) of radius r on a cubic grid with uniform
                   jitter of the centres
  chains           n random-walk chains of m markers, bond length b,
                   starts uniform
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 20261200


def rng(index: int) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + index)


def _unit(g: np.random.Generator, n: int) -> np.ndarray:
    v = g.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def stokeslet_box(L: int = 32, index: int = 1):
    g = rng(index)
    pos = g.uniform(0, L, size=(1, 3))
    force = np.array([[0.0, 0.0, 1e-5]])
    return pos, force


def singularities(L: int = 128, n: int = 64, index: int = 2, smax: float = 1e-5, sep: float = 2.0):
    g = rng(index)
    types = g.integers(0, 3, size=n).astype(np.int32)
    centers = g.uniform(0, L, size=(n, 3))
    axes = _unit(g, n)
    e1 = g.normal(size=(n, 3))
    e1 -= axes * (e1 * axes).sum(1, keepdims=True)
    e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    strengths = g.uniform(-smax, smax, size=n)
    return dict(types=types, centers=centers, axes=axes, e1=e1, strengths=strengths, sep=sep)


def colloids(L: int, n: int, index: int = 3, fz: float = -1e-6, shape=None):
    g = rng(index)
    ext = np.array(shape[::-1] if shape is not None else (L, L, L), dtype=np.float64)
    pos = g.uniform(0, 1, size=(n, 3)) * ext
    force = np.tile([0.0, 0.0, fz], (n, 1))
    return pos, force


def mobility_boxes(nboxes: int = 512, L: int = 32, index: int = 4, fz: float = -1e-6, kmax: int = 8,
                   tau_range=(0.6, 1.5)):
    g = rng(index)
    counts = g.integers(1, kmax + 1, size=nboxes)
    taus = g.uniform(tau_range[0], tau_range[1], size=nboxes)
    pos, box, off = [], [], []
    h = L // 2
    for b in range(nboxes):
        for j in range(int(counts[b])):
            o = g.uniform(0, 1, size=3)
            site = np.array([h // 2 + h * (j & 1), h // 2 + h * ((j >> 1) & 1), h // 2 + h * (j >> 2)], float)
            pos.append(site + o)
            off.append(o)
            box.append(b)
    pos = np.array(pos)
    force = np.tile([0.0, 0.0, fz], (len(pos), 1))
    return dict(pos=pos, force=force, box=np.array(box, dtype=np.int32), offsets=np.array(off),
                counts=counts, taus=taus)


def geodesic_sphere(levels: int):
    """Unit-sphere triangulation: an icosahedron subdivided `levels` times, vertices projected to
    the sphere, triangles counter-clockwise seen from outside (geometry only)."""
    t = (1 + 5 ** 0.5) / 2
    verts = [np.array(v, dtype=np.float64) / np.linalg.norm(v) for v in
             ((-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
              (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1))]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
             (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5), (2, 4, 11),
             (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(levels):
        mids = {}

        def mid(i, j):
            k = (min(i, j), max(i, j))
            if k not in mids:
                m = verts[i] + verts[j]
                verts.append(m / np.linalg.norm(m))
                mids[k] = len(verts) - 1
            return mids[k]

        faces = [f for a, b, c in faces for f in ((a, mid(a, b), mid(c, a)), (b, mid(b, c), mid(a, b)),
                                                   (c, mid(c, a), mid(b, c)), (mid(a, b), mid(b, c), mid(c, a)))]
    V = np.array(verts)
    F = np.array(faces, dtype=np.int32)
    n = np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]])
    flip = (n * V[F].mean(1)).sum(1) < 0
    F[flip] = F[flip][:, [0, 2, 1]]
    return V, F


def droplets(L: int, n: int, radius: float, levels: int = 3, index: int = 5):
    """n spheres of the given radius on the sites of a cubic grid filling the box, centres jittered
    by U[-1/2, 1/2)^3; returns (positions, triangles) of one combined marker set."""
    g = rng(index)
    k = int(np.ceil(n ** (1 / 3)))
    sp = L / k
    V, F = geodesic_sphere(levels)
    pos, tri = [], []
    for j in range(n):
        site = np.array([j % k, (j // k) % k, j // (k * k)], dtype=np.float64)
        c = (site + 0.5) * sp + g.uniform(-0.5, 0.5, 3)
        pos.append(c + radius * V)
        tri.append(F + j * len(V))
    return np.concatenate(pos), np.concatenate(tri)


def chains(L: int, n: int, m: int, bond: float = 1.0, index: int = 6):
    """n chains of m markers: uniform starts, steps of length `bond` in uniform directions."""
    g = rng(index)
    start = g.uniform(0, L, (n, 1, 3))
    steps = _unit(g, n * (m - 1)).reshape(n, m - 1, 3) * bond
    pos = np.concatenate([start, start + np.cumsum(steps, axis=1)], axis=1).reshape(-1, 3)
    return pos - L * np.floor(pos / L)
