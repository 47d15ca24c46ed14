"""Autotuner for the fused step kernel: tile shape x access variant.

    python -m paper_0707_1299_amd.tune --shape 128 128 128 --storage fp32 [--nboxes 1]
                                      [--points singularities|colloids|boxes --npoints N]

For each candidate it builds a context with the workload's points, warms
up, times whole steps (wall clock, graph replay) and the fused kernel alone
(HIP events, lb_kernel_timing), and keeps the fastest whole step.  Results are
cached per (arch, storage, box shape, box count) in tune_cache.json next to
this file; ``lookup`` returns the cached choice or None.  Every candidate
computes identical results (the parity tests check that bit for bit), so the
choice only affects speed.
"""
from __future__ import annotations

import argparse
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tune_cache.json")
ARCH = "gfx950"
TILES = [(64, 2, 2), (64, 4, 1), (64, 1, 4), (128, 2, 1), (128, 1, 2), (256, 1, 1), (32, 4, 2), (32, 2, 4),
         (16, 4, 4)]
VARIANTS = [0, 2, 4, 6, 8, 10, 16, 18, 20, 22, 66, 70]
# the one-tile-per-block variants also in the step kernel built without the tile loop (bit 128)
VARIANTS += [v | 128 for v in VARIANTS if not (v >> 2) & 3]


def key(shape, storage, nboxes, tag=None):
    nz, ny, nx = shape
    k = "%s/%s/%dx%dx%d/b%d" % (ARCH, storage, nx, ny, nz, nboxes)
    return k + "/" + tag if tag else k


def lookup(shape, storage, nboxes=1, tag=None):
    """(tile, variant) cached for this shape and storage; with a tag (a named workload, whose
    points or collision options change the best choice) the tagged entry if there is one."""
    if not os.path.exists(CACHE):
        return None
    c = json.load(open(CACHE))
    d = (c.get(key(shape, storage, nboxes, tag)) if tag else None) or c.get(key(shape, storage, nboxes))
    if not d:
        return None
    return tuple(d["tile"]), int(d["variant"])


def save(shape, storage, nboxes, entry, tag=None):
    d = json.load(open(CACHE)) if os.path.exists(CACHE) else {}
    d[key(shape, storage, nboxes, tag)] = entry
    with open(CACHE, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)


PLANES = {"fp64": 19, "fp32": 19, "fp16": 19, "mom32": 10}
ELEM_BYTES = {"fp64": 8, "fp32": 4, "fp16": 2, "mom32": 4}


def candidates(shape, storage="fp32"):
    nz, ny, nx = shape
    # tiles with fewer than 64 lanes along x need boxes under 4 GiB; FP16 with nx even runs two
    # nodes per lane
    big = nx * ny * nz * PLANES[storage] * ELEM_BYTES[storage] >= 4.0e9
    npl = 2 if storage == "fp16" and nx % 2 == 0 else 1
    out = []
    for t in TILES:
        for v in VARIANTS + ([v | 32 for v in VARIANTS] if npl == 2 else []):
            lanes = t[0] // (1 if v & 32 else npl)        # bit 32: one FP16 node per lane
            if t[0] > 2 * nx or (big and lanes < 64):
                continue
            if v & 64 and nx // t[0] < 2 * (1 << ((v >> 2) & 3)):
                continue        # one run per tile row: the same block order as launch order
            out.append((t, v))
    return out


def make_points(kind, shape, n, nboxes=1):
    """Seeded points of a workload: 'singularities' (static multipoles), 'colloids' (advected) or
    'boxes' (fixed colloids, one set per box)."""
    import numpy as np
    from . import lbm, workloads
    if kind == "singularities":
        w = workloads.singularities(L=shape[2], n=n)
        pos, frc = lbm.lb_expand_multipoles(w["types"], w["centers"], w["axes"], w["e1"], w["strengths"], w["sep"])
        return dict(pos=pos, force=frc, box=None, kind=lbm.LB_FORCES_STATIC, model=None, zero_net=False)
    if kind == "colloids":
        pos, frc = workloads.colloids(shape[2], n, shape=shape)
        return dict(pos=pos, force=frc, box=None, kind=lbm.LB_COLLOIDS,
                    model=dict(inv_a=1 / 0.117, inv_aL=0.77), zero_net=True)
    if kind == "boxes":
        w = workloads.mobility_boxes(nboxes=nboxes, L=shape[2])
        return dict(pos=w["pos"], force=w["force"], box=w["box"], kind=lbm.LB_FORCES_STATIC, model=None,
                    zero_net=True, taus=w["taus"])
    return None


def measure(shape, storage, nboxes, tile, variant, steps, points):
    """(fused-kernel ms, whole-step ms) for one candidate."""
    import time
    import torch
    from . import lbm
    pts = points or {}
    npts = len(pts.get("pos", ()))
    lat = lbm.Lattice(shape, storage, nboxes=nboxes, tau=pts.get("taus", 0.5), max_points=max(1, npts), tile=tile,
                      variant=variant, zero_net_force=pts.get("zero_net", False))
    if npts:
        model = lbm.PointModel(**pts["model"]) if pts.get("model") else None
        box = None if pts.get("box") is None else torch.tensor(pts["box"], dtype=torch.int32, device="cuda")
        lat.add_point_forces(torch.tensor(pts["pos"], device="cuda"), torch.tensor(pts["force"], device="cuda"),
                             box, pts["kind"], model)
    lat.step(10)
    lat.prepare_steps(steps)     # graph capture outside the timed call
    lat.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.step(steps)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps * 1e3
    lat.kernel_timing(True)
    lat.step(max(5, steps // 2))
    ms, n = lat.kernel_time()
    lat.close()
    return ms / n, wall


def tune(shape, storage, nboxes=1, steps=100, points=None, save=True, verbose=True):
    """Sweep the candidates; the choice minimises the whole-step time (the fused kernel plus
    the point pipeline, which depends on how many tiles a point's stencil touches)."""
    N = shape[0] * shape[1] * shape[2] * nboxes
    bpn = {"fp64": 304, "fp32": 152, "fp16": 76, "mom32": 80}[storage]
    res = []
    for tile, variant in candidates(shape, storage):
        ms, wall = measure(shape, storage, nboxes, tile, variant, steps, points)
        gbs = bpn * N / (ms * 1e-3) / 1e9
        res.append(dict(tile=list(tile), variant=variant, kernel_ms=ms, step_ms=wall, GBs=gbs))
        if verbose:
            print("tile %-14s variant %d  kernel %.4f ms (%.1f GB/s)  step %.4f ms" % (tile, variant, ms, gbs, wall),
                  flush=True)
    best = min(res, key=lambda r: r["step_ms"])
    if save:
        globals()["save"](shape, storage, nboxes, dict(tile=best["tile"], variant=best["variant"],
                                                       kernel_ms=best["kernel_ms"], step_ms=best["step_ms"],
                                                       GBs=best["GBs"]))
    return best, res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--shape", type=int, nargs=3, default=[128, 128, 128], help="nz ny nx")
    ap.add_argument("--storage", default="fp32")
    ap.add_argument("--nboxes", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--points", default=None, help="singularities | colloids | boxes")
    ap.add_argument("--npoints", type=int, default=64)
    a = ap.parse_args()
    pts = make_points(a.points, tuple(a.shape), a.npoints, a.nboxes) if a.points else None
    best, _ = tune(tuple(a.shape), a.storage, a.nboxes, a.steps, points=pts)
    print(json.dumps(best))


if __name__ == "__main__":
    main()
