"""Write the FP64 oracle's results for the long runs of two workloads, sampled,
to tests/golden/ (TEST INFRASTRUCTURE: calls only the oracle and the seeded
input generators).

    python tests/golden/make_long_goldens.py [singularities128] [colloids256]

  singularities128  128^3 periodic box, tau = 1/2, 64 seeded singularities
                    (Stokeslets, stresslets, rotlets; |s| <= 1e-5, separation
                    2) as their point forces, static, counter-force off,
                    5000 steps (the full stated length of that workload);
  colloids256       256^3 periodic box, tau = 1/2, 10^4 sedimenting colloids
                    (F = -1e-6 z, a = 0.117, 1/a_L = 0.77), counter-force on,
                    1000 steps.

Each file holds, after the last step:
  * the physical velocity u and density rho (Eq. macrovariables2) at sampled
    nodes: the 2x2x2 nodes around each of the force points (or of a seeded
    sample of 512 colloids at their final positions) and 2048 uniform nodes;
  * max |u| over every node and component (the denominator of the relative
    error norm of the parity tests);
  * the interpolated velocity U of the last step and the positions (all force
    points, or a seeded sample of 2048 colloids);
  * per population the sum over the lattice of the pre-collision deviation
    (total mass and auxiliary momentum, Eq. conservation);
  * the sha256 of the oracle's C source, so that a stale file is detected.

A run takes about 45 minutes (singularities128) and one hour (colloids256) on
8 host threads.
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import multipole  # noqa: E402
from paper_0707_1299_amd import workloads  # noqa: E402  (seeded random draws only)

SAMPLE_SEED = 20261290
WORKLOADS = {
    "singularities128": dict(L=128, steps=5000, tau=0.5),
    "colloids256": dict(L=256, n=10000, steps=1000, tau=0.5, a=0.117, inv_aL=0.77),
}


def oracle_source_sha():
    h = hashlib.sha256()
    h.update(open(os.path.join(ROOT, "oracle", "lbm_oracle.c"), "rb").read())
    return h.hexdigest()


def node_sample(shape, pts, g, n_uniform=2048):
    """Flat node indices: the 2x2x2 nodes around each point, then n_uniform uniform nodes."""
    nz, ny, nx = shape
    base = np.floor(pts).astype(np.int64)
    idx = []
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                x = (base[:, 0] + dx) % nx
                y = (base[:, 1] + dy) % ny
                z = (base[:, 2] + dz) % nz
                idx.append((z * ny + y) * nx + x)
    near = np.unique(np.concatenate(idx))
    uni = g.integers(0, nx * ny * nz, size=n_uniform)
    return np.unique(np.concatenate([near, uni]))


def finish(name, box, pts_for_nodes, g, extra):
    shape = box.shape
    rho, u = box.moments()
    nodes = node_sample(shape, pts_for_nodes, g)
    uf = u.reshape(3, -1)
    c, _ = oracle.velocities()
    dfsum = box.df.reshape(19, -1).sum(axis=1)
    out = dict(nodes=nodes, u=uf[:, nodes].copy(), rho=rho.reshape(-1)[nodes].copy(),
               umax=np.abs(u).max(), df_sum=dfsum, c=c, steps=box.steps, tau=box.tau,
               oracle_sha=np.array(oracle_source_sha()), threads=oracle.threads(), **extra)
    path = os.path.join(HERE, "%s_oracle_%d.npz" % (name, box.steps))
    np.savez_compressed(path, **out)
    print("wrote %s (%d sampled nodes, max|u| %.4e)" % (path, len(nodes), out["umax"]), flush=True)


def run(name):
    w = WORKLOADS[name]
    L, steps = w["L"], w["steps"]
    g = np.random.default_rng(SAMPLE_SEED)
    t0 = time.time()
    if name == "singularities128":
        s = workloads.singularities(L=L, n=64)
        pos, frc = multipole.expand(s["types"], s["centers"], s["axes"], s["e1"], s["strengths"], s["sep"])
        box = oracle.Box((L, L, L), w["tau"], 1.0, zero_net_force=False)
        box.sets = [oracle.ForceSet(pos, frc)]
    else:
        pos, frc = workloads.colloids(L, w["n"])
        box = oracle.Box((L, L, L), w["tau"], 1.0, zero_net_force=True)
        box.sets = [oracle.ForceSet(pos.copy(), frc.copy(), kind="colloid", inv_a=1 / w["a"], inv_aL=w["inv_aL"])]
    done = 0
    while done < steps:
        k = min(50, steps - done)
        box.step(k)
        done += k
        print("%s: %d/%d steps, %.0f s" % (name, done, steps, time.time() - t0), flush=True)
    fs = box.sets[0]
    if name == "singularities128":
        finish(name, box, fs.pos, g, dict(U=fs.U.copy(), pos=fs.pos.copy()))
    else:
        pick = np.sort(g.choice(len(fs.pos), size=2048, replace=False))
        near = np.sort(g.choice(len(fs.pos), size=512, replace=False))
        finish(name, box, fs.pos[near], g, dict(pick=pick, U=fs.U[pick].copy(), pos=fs.pos[pick].copy(),
                                                pos0=pos[pick].copy()))


if __name__ == "__main__":
    for n in (sys.argv[1:] or list(WORKLOADS)):
        run(n)
