"""Benchmark: throughput of the forced D3Q19 step with spread / interpolated
point forces on one MI355X, with the dominant kernel's HBM roofline and the
FP64 CPU oracle timed beside it.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload NAME] [--no-cpu]

Default (--workload headline): the 512^3 periodic lattice with 10^5
sedimenting point colloids (F = -1e-6 z, a = 0.684, volume fraction ~1e-3,
tau = 1/2, counter-force on), spread + step + interpolate + advect every step,
in two forms:
  * plain: FP32 deviation storage, the constant 1/a_L fitted for tau = 1/2
    (`value`, the fused kernel's `roofline`);
  * chosen: FP16-scaled storage and the trained mobility network
    (paper_0707_1299_amd/mobility_net.json) in the colloid update
    (`chosen_form`, with its own roofline);
with the colloid updates per second of both, the mobility error of both
against single-particle full-lattice runs at tau = 1/2, the error of both
against the FP64 oracle after a few steps, and the oracle's own rate on the
same 512^3 workload (`cpu_baseline`).  Other workloads: --workload NAME.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0          # MI355X HBM3E
# read + write of one node's stored state: 19 populations (fp64/fp32/fp16) or 10 FP32 moments
BYTES_PER_NODE = {"fp64": 304, "fp32": 152, "fp16": 76, "mom32": 80}

WORKLOADS = {
    # name: (shape, storage, tau, kind, n)
    "singularities128": ((128, 128, 128), "fp32", 0.5, "singularities", 64),
    "boxes512x32_fp32": ((32, 32, 32), "fp32", None, "boxes", 512),
    "boxes512x32_fp16": ((32, 32, 32), "fp16", None, "boxes", 512),
    "colloids256_fp32": ((256, 256, 256), "fp32", 0.5, "colloids", 10000),
    "colloids256_fp16": ((256, 256, 256), "fp16", 0.5, "colloids", 10000),
    "colloids256_fp64": ((256, 256, 256), "fp64", 0.5, "colloids", 10000),
    "colloids512_fp32": ((512, 512, 512), "fp32", 0.5, "colloids", 100000),
    "colloids512_fp16": ((512, 512, 512), "fp16", 0.5, "colloids", 100000),
    "singularities128_mom32": ((128, 128, 128), "mom32", 0.5, "singularities", 64),
    "boxes512x32_mom32": ((32, 32, 32), "mom32", None, "boxes", 512),
    "colloids256_mom32": ((256, 256, 256), "mom32", 0.5, "colloids", 10000),
    "colloids512_mom32": ((512, 512, 512), "mom32", 0.5, "colloids", 100000),
    "singularities128_bgk": ((128, 128, 128), "fp32", 0.5, "singularities", 64),
    "singularities128_mrt": ((128, 128, 128), "fp32", 0.5, "singularities", 64),
    "singularities128_fp16_bgk": ((128, 128, 128), "fp16", 0.5, "singularities", 64),
    "singularities128_thermal": ((128, 128, 128), "fp32", 0.5, "singularities", 64),
    "colloids256_thermal": ((256, 256, 256), "fp32", 0.5, "colloids", 10000),
    "droplets256": ((256, 256, 256), "fp32", 0.8, "droplets", 64),
    "chains256": ((256, 256, 256), "fp32", 0.8, "chains", 2048),
    # one GPU's share of the 512^3 lattice split into 8 z-slabs (10^5 / 8 colloids), periodic in z
    "slab512x512x64_fp32": ((64, 512, 512), "fp32", 0.5, "slab", 12500),
    "slab512x512x64_fp16": ((64, 512, 512), "fp16", 0.5, "slab", 12500),
}
# lattice options of a workload: collision operator (default: the projected operator of
# Eq. fiexp) and thermal noise
OPTS = {
    "singularities128_bgk": dict(collision="bgk"),
    "singularities128_mrt": dict(collision="mrt", tau_bulk=1.0, ghost_rate=1.5),
    "singularities128_fp16_bgk": dict(collision="bgk"),
    "singularities128_thermal": dict(kT=1e-5, seed=7),
    "colloids256_thermal": dict(kT=1e-5, seed=7),
}
DESCR = {
    "singularities": "%d^3 periodic D3Q19 forced MRT, %s deviation storage, tau=1/2, %d seeded point "
                     "singularities (Stokeslet/stresslet/rotlet, |s|<=1e-5) as %d point forces",
    "colloids": "%d^3 periodic D3Q19 forced MRT, %s storage, tau=1/2, %d sedimenting point colloids "
                "(F=-1e-6 z, a=0.117 at 256^3, 0.684 at 512^3), spread + interpolate + advect every step, "
                "counter-force on",
    "boxes": "%d independent %d^3 boxes in one context, %s storage, tau_b ~ U[0.6,1.5], 1-8 fixed colloids "
             "per box (%d total), counter-force on, interpolated velocity accumulated every step",
    "droplets": "%d^3 periodic D3Q19 forced MRT, %s storage, tau=0.8, %d triangulated droplet interfaces "
                "(R=12, 642 markers each, tension 1e-4): marker forces, spread, interpolate, move every step",
    "chains": "%d^3 periodic D3Q19 forced MRT, %s storage, tau=0.8, %d bead-spring chains of 32 markers "
              "(k=1e-3, l0=1, F_ext=-1e-6 z), counter-force on: marker forces, spread, interpolate, move every step",
    "slab": "%dx%dx%d slab (one GPU's share of a 512^3 lattice in 8 z-slabs; periodic wrap in z standing in for "
            "the halo exchange), %s storage, tau=1/2, %d sedimenting point colloids (a=0.684), counter-force on",
}


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("lbm_lattice_impl.h", "lbm_device.h", "lbm_noise.h", "lbm_api.hip"):
        h.update(open(os.path.join(ROOT, "paper_0707_1299_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def make_inputs(kind, shape, n):
    import numpy as np
    from paper_0707_1299_amd import lbm, workloads
    L = shape[0]
    if kind == "boxes":
        w = workloads.mobility_boxes(nboxes=n, L=L)
        return w, None, "boxes", None
    if kind == "singularities":
        w = workloads.singularities(L=L, n=n)
        pos, frc = lbm.lb_expand_multipoles(w["types"], w["centers"], w["axes"], w["e1"], w["strengths"], w["sep"])
        return pos, frc, "static", None
    if kind == "droplets":
        pos, tri = workloads.droplets(L, n, radius=12.0, levels=3)
        return dict(pos=pos, tri=tri, tension=1e-4), None, "droplets", None
    if kind == "chains":
        pos = workloads.chains(L, n, 32)
        ext = np.tile([0.0, 0.0, -1e-6], (len(pos), 1))
        return dict(pos=pos, ext=ext, chain_len=32, k=1e-3, l0=1.0), None, "chains", None
    if kind == "slab":
        pos, frc = workloads.colloids(shape[2], n, shape=shape)
        return pos, frc, "colloid", dict(inv_a=1 / 0.684, inv_aL=0.77)
    pos, frc = workloads.colloids(L, n)
    # a = 0.117 (Table 1) at 256^3 with 1/a_L = 0.77; a = 0.684 (volume fraction ~1e-3 with 10^5
    # colloids) at 512^3 with the plain 1/a_L fitted for the run's tau
    if L >= 512:
        return pos, frc, "colloid", dict(inv_a=1 / 0.684, inv_aL=None)
    return pos, frc, "colloid", dict(inv_a=1 / 0.117, inv_aL=0.77)


def point_model(model, tau):
    """The colloid model of a workload: model["mlp"] True uses the trained network
    (mobility_net.json) in the update; model["inv_aL"] None the plain constant fitted for tau."""
    from paper_0707_1299_amd import lbm, mobility
    if model.get("mlp") or model.get("inv_aL") is None:
        tr = mobility.load(mobility.DEFAULT_NET)
        if model.get("mlp"):
            return tr.model(model["inv_a"])
        return tr.plain_model(model["inv_a"], tau)
    return lbm.PointModel(inv_a=model["inv_a"], inv_aL=model["inv_aL"])


def tuned(shape, storage, nboxes=1, tag=None):
    from paper_0707_1299_amd import tune
    return tune.lookup(shape, storage, nboxes, tag) or (None, 0)


def build_lattice(shape, storage, tau, kind, pos, frc, model, opts=None, name=None, choice=None):
    """The workload's lattice and points; tile and variant from `choice` or the tuning cache."""
    import torch
    from paper_0707_1299_amd import lbm
    opts = opts or {}
    if kind == "boxes":
        w = pos
        nb = len(w["taus"])
        tile, variant = choice or tuned(shape, storage, nb, name)
        lat = lbm.Lattice(shape, storage, nboxes=nb, tau=w["taus"], zero_net_force=True, max_points=len(w["pos"]),
                          tile=tile, variant=variant, **opts)
        p = torch.tensor(w["pos"], dtype=torch.float64, device="cuda")
        vsum = torch.zeros_like(p)
        lat.add_point_forces(p, torch.tensor(w["force"], dtype=torch.float64, device="cuda"),
                             torch.tensor(w["box"], dtype=torch.int32, device="cuda"), lbm.LB_FORCES_STATIC,
                             lbm.PointModel(vel_sum=vsum))
        return lat, p
    tile, variant = choice or tuned(shape, storage, 1, name)
    if kind in ("droplets", "chains"):
        w = pos
        lat = lbm.Lattice(shape, storage, tau=tau, zero_net_force=(kind == "chains"), max_points=len(w["pos"]),
                          tile=tile, variant=variant, **opts)
        p = torch.tensor(w["pos"], dtype=torch.float64, device="cuda")
        if kind == "droplets":
            lat.add_surface(p, w["tri"], w["tension"])
        else:
            lat.add_chains(p, w["chain_len"], w["k"], w["l0"],
                           ext=torch.tensor(w["ext"], dtype=torch.float64, device="cuda"))
        return lat, p
    lat = lbm.Lattice(shape, storage, tau=tau, zero_net_force=(kind == "colloid"), max_points=len(pos), tile=tile,
                      variant=variant, **opts)
    p = torch.tensor(pos, dtype=torch.float64, device="cuda")
    f = torch.tensor(frc, dtype=torch.float64, device="cuda")
    if kind == "colloid":
        lat.add_point_forces(p, f, None, lbm.LB_COLLOIDS, point_model(model, tau))
    else:
        lat.add_point_forces(p, f, None, lbm.LB_FORCES_STATIC)
    return lat, p


def traffic_from_profile(name, storage, N, record=None):
    """HBM bytes per launch from the committed rocprofv3 counter summary (profiles/traffic_<record or
    name>.json), if it was taken on the current kernel source and launch choice; else None."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % (record or name))
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("kernel_sha") != kernel_source_hash():
        return None
    shape = WORKLOADS[name][0]
    tile, variant = tuned(shape, storage, WORKLOADS[name][4] if WORKLOADS[name][3] == "boxes" else 1, name)
    if list(tile or []) != d.get("tile") or variant != d.get("variant"):
        return None
    return d.get("bytes_per_launch")


def oracle_model(model, tau):
    """(inv_a, inv_aL, inv_aL_fn) of the oracle's colloid update for a workload's model: the same
    constant, or the same bf16 network evaluated in FP64."""
    if not model:
        return 0.0, 0.0, None
    pm = point_model(model, tau)
    if not model.get("mlp"):
        return pm.inv_a, pm.inv_aL, None
    import numpy as np
    from oracle import mlp as omlp
    from paper_0707_1299_amd import mobility
    tr = mobility.load(mobility.DEFAULT_NET)
    theta = mobility.weights_f64(tr)

    def inv_aL_fn(p, t):
        o = p - np.floor(p)
        y, _ = omlp.forward(theta, mobility.features(o, np.full(len(p), t)), round_bf16=False)
        return tr.mu_plain + tr.out_scale * y

    return pm.inv_a, pm.inv_aL, inv_aL_fn


def cpu_baseline(kind, shape, storage, tau, pos, frc, model, budget_s=12.0, max_steps=200):
    """The FP64 oracle, as it is, on a bounded number of steps of the same workload."""
    import numpy as np
    import oracle
    box = oracle.Box(shape, tau, 1.0, zero_net_force=(kind == "colloid"))
    inv_a, inv_aL, fn = oracle_model(model, tau) if kind == "colloid" else (0.0, 0.0, None)
    fs = oracle.ForceSet(np.array(pos), np.array(frc), kind=kind, inv_a=inv_a, inv_aL=inv_aL, inv_aL_fn=fn)
    box.sets = [fs]
    t0 = time.perf_counter()
    box.step(1)
    t1 = time.perf_counter()
    per = t1 - t0
    steps = int(max(1, min(max_steps, budget_s / max(per, 1e-6))))
    t0 = time.perf_counter()
    box.step(steps)
    dt = time.perf_counter() - t0
    N = shape[0] * shape[1] * shape[2]
    return box, steps + 1, dict(value=round(N * steps / dt / 1e6, 3), unit="MLUPS", cores=oracle.threads(),
                                kind="oracle",
                                sample="steps 2..%d of the same workload (%d steps, %.1f s), FP64, OpenMP"
                                       % (steps + 1, steps, dt))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def oracle_rates():
    """The FP64 oracle on bounded samples of the other configurations, all host threads and one:
    32^3 Stokeslet, 256^3 with 10^4 colloids, 512^3 with 10^5 colloids (2 steps), and the
    128^3 singularities box on one thread."""
    import oracle
    from paper_0707_1299_amd import workloads
    out = {"cpu": cpu_model(), "threads": oracle.threads()}
    pos, frc = workloads.stokeslet_box(32)
    _, _, cb = cpu_baseline("static", (32, 32, 32), "fp64", 0.5, pos, frc, None, budget_s=5.0)
    out["stokeslet32_fp64"] = cb
    for L, n, budget in ((256, 10000, 10.0), (512, 100000, 1.0)):
        pos, frc, fkind, model = make_inputs("colloids", (L, L, L), n)
        _, _, cb = cpu_baseline(fkind, (L, L, L), "fp64", 0.5, pos, frc, model, budget_s=budget)
        out["colloids%d" % L] = cb
        print("oracle %d^3 done" % L, file=sys.stderr, flush=True)
    nthr = oracle.threads()
    oracle.set_threads(1)
    pos, frc, fkind, model = make_inputs("singularities", (128, 128, 128), 64)
    _, _, cb = cpu_baseline(fkind, (128, 128, 128), "fp64", 0.5, pos, frc, model, budget_s=8.0)
    oracle.set_threads(nthr)
    out["singularities128_one_thread"] = cb
    return out


def run_workload(name, steps, warmup, timing_steps, mlp=False, choice=None):
    """Time one workload; returns (result dict, inputs) for the JSON line."""
    import torch
    shape, storage, tau, kind, n = WORKLOADS[name]
    nb = n if kind == "boxes" else 1
    N = shape[0] * shape[1] * shape[2] * nb
    pos, frc, fkind, model = make_inputs(kind, shape, n)
    if mlp and model is not None:
        model = dict(model, mlp=True)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        lat, dpos = build_lattice(shape, storage, tau, fkind, pos, frc, model, OPTS.get(name), name, choice)
        lat.step(warmup)
        # graphs of the timed call's chunk lengths captured now (no step taken), not while timed
        lat.prepare_steps(steps)
        lat.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat.step(steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        lat.sync()
        elapsed = t1 - t0
        # dominant kernel: HIP events around every fused-step launch on this stream
        lat.kernel_timing(True)
        lat.step(timing_steps)
        ktot_ms, nlaunch = lat.kernel_time()
        lat.kernel_timing(False)
        lat.close()
    kavg_s = ktot_ms / nlaunch / 1e3
    achieved = BYTES_PER_NODE[storage] * N / kavg_s / 1e9
    npts = len(pos["pos"]) if kind in ("boxes", "droplets", "chains") else len(pos)
    r = dict(mlups=N * steps / elapsed / 1e6, ms_per_step=elapsed / steps * 1e3, kernel_ms=kavg_s * 1e3,
             achieved_GBs=achieved, frac=achieved / PEAK_HBM_GBS, nodes=N, points=int(npts), storage=storage,
             launches_timed=nlaunch, steps=steps)
    if kind in ("colloid", "colloids", "slab"):
        r["colloid_updates_per_s"] = n * steps / elapsed
    if kind in ("boxes", "droplets", "chains"):
        r["point_updates_per_s"] = npts * steps / elapsed
    return r, (shape, storage, tau, kind, n, pos, frc, fkind, model)


def tune_workload(name, steps=40, refine=5):
    """Every candidate (tile, variant) of the tuner on this workload as it is timed (its points,
    markers, collision options), then the `refine` fastest again over 5x the steps (short runs
    differ by a few per cent from run to run); the fastest whole step of the second pass is
    cached under the workload's name."""
    from paper_0707_1299_amd import tune
    shape, storage, tau, kind, n = WORKLOADS[name]
    nb = n if kind == "boxes" else 1

    def timed(tile, variant, k):
        r, _ = run_workload(name, k, 10, max(5, k // 2), choice=(tile, variant))
        return dict(tile=list(tile), variant=variant, kernel_ms=r["kernel_ms"], step_ms=r["ms_per_step"],
                    GBs=r["achieved_GBs"])

    res = []
    for tile, variant in tune.candidates(shape, storage):
        res.append(timed(tile, variant, steps))
        print("tile %-14s variant %2d  kernel %.4f ms  step %.4f ms" % (tile, variant, res[-1]["kernel_ms"],
                                                                        res[-1]["step_ms"]), flush=True)
    top = sorted(res, key=lambda e: e["step_ms"])[:refine]
    final = []
    for e in top:
        final.append(timed(tuple(e["tile"]), e["variant"], 5 * steps))
        print("refine tile %-14s variant %2d  kernel %.4f ms  step %.4f ms" % (
            tuple(e["tile"]), e["variant"], final[-1]["kernel_ms"], final[-1]["step_ms"]), flush=True)
    best = min(final, key=lambda e: e["step_ms"])
    tune.save(shape, storage, nb, best, tag=name)
    print(json.dumps(dict(best, workload=name)))


def stream_copy_gbs(nbytes, reps=20):
    """Measured HBM copy rate (read + write bytes / time, GB/s) of the library's streaming-copy probe
    over nbytes, timed with HIP events on the stream it runs on: the practical ceiling a streaming
    kernel is set against beside the vendor peak."""
    import torch
    from paper_0707_1299_amd import lbm
    nbytes = (nbytes + 15) // 16 * 16
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        lbm.lb_copy_probe(src, dst)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        lbm.lb_copy_probe(src, dst)
    e1.record()
    torch.cuda.synchronize()
    assert bool(torch.equal(src, dst))
    gbs = 2 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def describe(name, r):
    shape, storage, tau, kind, n = WORKLOADS[name]
    if kind == "singularities":
        d = DESCR[kind] % (shape[0], storage, n, r["points"])
    elif kind == "boxes":
        d = DESCR[kind] % (n, shape[0], storage, r["points"])
    elif kind == "slab":
        d = DESCR[kind] % (shape[2], shape[1], shape[0], storage, n)
    else:
        d = DESCR[kind] % (shape[0], storage, n)
    c = OPTS.get(name)
    if c:
        d += ", %s" % ", ".join("%s=%s" % kv for kv in sorted(c.items()))
    return d


def roofline(r, storage, traffic, copy_gbs=None, copy_same_gbs=None):
    """The fused step kernel's HBM roofline entry for one timed workload."""
    d = {"bound": "hbm", "achieved": round(r["achieved_GBs"], 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
         "frac": round(r["frac"], 4), "traffic": traffic,
         "kernel": "k_lattice step (fused spread/pull/collide/store/interpolate)",
         "bytes_per_node": BYTES_PER_NODE[storage], "kernel_ms": round(r["kernel_ms"], 5),
         "launches_timed": r["launches_timed"]}
    if copy_gbs:
        d.update(copy_1GiB_GBs=round(copy_gbs, 1), frac_of_copy=round(r["achieved_GBs"] / copy_gbs, 4))
    if copy_same_gbs:
        d.update(copy_same_bytes_GBs=round(copy_same_gbs, 1),
                 frac_of_copy_same_bytes=round(r["achieved_GBs"] / copy_same_gbs, 4))
    return d


def mobility_error(n=128, tau=0.5, L=32):
    """Self-mobility error of the plain constant (fitted for tau) and of constant + network, against
    fresh single-particle full-lattice runs (one fixed colloid per 32^3 box, 2000 steps, the last 200
    averaged) at seeded offsets the network was not trained on."""
    import numpy as np
    from paper_0707_1299_amd import mobility, workloads
    tr = mobility.load(mobility.DEFAULT_NET)
    off = workloads.rng(8).uniform(0, 1, size=(n, 3))
    taus = np.full(n, tau)
    mu = mobility.self_part(mobility.single_particle_labels(off, taus, L=L, steps=2000, average=200), L)
    ev = mobility.evaluate(tr, off, taus, mu)
    return {"reference": "%d single-particle %d^3 runs at tau=%g (fixed colloid, 2000 steps, U averaged over the "
                         "last 200), seeded offsets not in the training set; mu = 6 pi eta U.F/|F|^2 + 2.84/L"
                         % (n, L, tau),
            "mu_mean": round(ev["mu_mean"], 5),
            "plain": {"rms": ev["rms_plain_tau"], "max": ev["max_plain_tau"], "inv_aL": float(tr.plain_tau(tau))},
            "mlp": {"rms": ev["rms_mlp"], "max": ev["max_mlp"]},
            "gain_rms": round(ev["rms_plain_tau"] / ev["rms_mlp"], 2)}


def oracle_error(name, csteps, box, model_over=None):
    """A fresh GPU run of the workload for csteps steps against the oracle box that ran them:
    velocity field, interpolated velocity and positions (relative to the oracle's displacement)."""
    import numpy as np
    import torch
    shape, storage, tau, kind, n = WORKLOADS[name]
    pos, frc, fkind, model = make_inputs(kind, shape, n)
    if model_over:
        model = dict(model, **model_over)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        lat, dpos = build_lattice(shape, storage, tau, fkind, pos, frc, model, OPTS.get(name), name)
        lat.step(csteps)
        _, u = lat.moments(rho=False)
        lat.sync()
        ug = u[0].cpu().numpy()
        Rg = dpos.cpu().numpy()
        lat.close()
    del u
    torch.cuda.empty_cache()
    _, uo = box.moments()
    out = {"steps": csteps, "velocity_rel_linf": float(np.abs(ug - uo).max() / np.abs(uo).max())}
    if fkind == "colloid":
        ext = np.array(shape[::-1], dtype=np.float64)
        d = np.abs(Rg - box.sets[0].pos)
        d = np.minimum(d, ext - d)
        m = np.abs(box.sets[0].pos - pos)
        m = np.minimum(m, ext - m)
        out["position_err_over_displacement"] = float(d.max() / m.max())
    return out


def headline(a):
    """The 512^3 workload with 10^5 colloids: plain FP32 (value) and FP16 + trained network."""
    import torch
    plain, chosen = "colloids512_fp32", "colloids512_fp16"
    r32, inp32 = run_workload(plain, a.steps, a.warmup, a.timing_steps)
    print("plain fp32 timed", file=sys.stderr, flush=True)
    r16, inp16 = run_workload(chosen, a.steps, a.warmup, a.timing_steps, mlp=True)
    print("fp16 + network timed", file=sys.stderr, flush=True)
    torch.cuda.empty_cache()
    copy_gbs = stream_copy_gbs(1 << 30)
    copy_same = stream_copy_gbs(BYTES_PER_NODE["fp32"] * r32["nodes"] // 2)
    shape = WORKLOADS[plain][0]
    t32, v32 = tuned(shape, "fp32", 1, plain)
    t16, v16 = tuned(shape, "fp16", 1, chosen)
    out = {
        "metric": "MLUPS and % HBM roofline; colloid updates/s vs plain FP32 at stated error",
        "value": round(r32["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(r32["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "512^3 periodic D3Q19 forced MRT, tau=1/2, 10^5 sedimenting point colloids (seeded "
                               "uniform positions, F=-1e-6 z, a=0.684, volume fraction ~1e-3), counter-force on; "
                               "spread + fused step + interpolate + advect every step. value: plain form (FP32 "
                               "deviation storage, constant 1/a_L fitted for tau=1/2)",
                   "nodes": r32["nodes"], "colloids": r32["points"], "seed": 20261203,
                   "tile": list(t32 or ()), "variant": v32},
        "roofline": roofline(r32, "fp32", traffic_from_profile(plain, "fp32", r32["nodes"]), copy_gbs, copy_same),
        "colloid_updates_per_s": round(r32["colloid_updates_per_s"], 1),
        "chosen_form": {
            "form": "FP16-scaled deviation storage (FP32 arithmetic) + trained 4-64-64-1 bf16 mobility network "
                    "in the colloid update",
            "mlups": round(r16["mlups"], 1), "ms_per_step": round(r16["ms_per_step"], 5),
            "colloid_updates_per_s": round(r16["colloid_updates_per_s"], 1),
            "speedup_vs_plain": round(r16["mlups"] / r32["mlups"], 4),
            "tile": list(t16 or ()), "variant": v16,
            "roofline": roofline(r16, "fp16", traffic_from_profile(chosen, "fp16", r16["nodes"], chosen + "_mlp"))},
    }
    out["mobility_error"] = mobility_error()
    print("mobility error leg done", file=sys.stderr, flush=True)
    if not a.no_cpu:
        shape, storage, tau, kind, n, pos, frc, fkind, model = inp32
        box, csteps, cb = cpu_baseline(fkind, shape, storage, tau, pos, frc, model, budget_s=10.0, max_steps=8)
        cb["sample"] += " (the 512^3 workload with 10^5 colloids, plain form)"
        out["cpu_baseline"] = cb
        errs = {"plain_fp32": oracle_error(plain, csteps, box)}
        del box
        print("oracle plain leg done", file=sys.stderr, flush=True)
        shape, storage, tau, kind, n, pos, frc, fkind, model = inp16
        import oracle
        inv_a, inv_aL, fn = oracle_model(dict(model, mlp=True), tau)
        box = oracle.Box(shape, tau, 1.0, zero_net_force=True)
        box.sets = [oracle.ForceSet(pos.copy(), frc.copy(), kind="colloid", inv_a=inv_a, inv_aL=inv_aL,
                                    inv_aL_fn=fn)]
        box.step(csteps)
        errs["chosen_fp16_mlp"] = oracle_error(chosen, csteps, box, dict(mlp=True))
        del box
        out["error_vs_oracle"] = errs
        out["oracle_cpu"] = cpu_model()
    return out


def all_workloads():
    """Every other workload, timed like the headline's forms (reported under 'workloads')."""
    extra = {}
    for name, steps, mlp in (("singularities128", 2000, False),
                             ("colloids256_fp32", 300, False), ("colloids256_fp16", 300, False),
                             ("colloids256_fp64", 200, False), ("colloids512_fp32", 100, False),
                             ("colloids512_fp16", 100, False), ("colloids512_fp16", 100, True),
                             ("boxes512x32_fp32", 300, False), ("boxes512x32_fp16", 300, False),
                             ("singularities128_mom32", 2000, False), ("colloids256_mom32", 300, False),
                             ("colloids512_mom32", 100, False), ("boxes512x32_mom32", 300, False),
                             ("singularities128_bgk", 2000, False), ("singularities128_mrt", 2000, False),
                             ("singularities128_fp16_bgk", 2000, False), ("singularities128_thermal", 2000, False),
                             ("colloids256_thermal", 300, False), ("droplets256", 300, False),
                             ("chains256", 300, False), ("slab512x512x64_fp32", 300, False),
                             ("slab512x512x64_fp16", 300, False)):
        rr, _ = run_workload(name, steps, 20, 50, mlp=mlp)
        rr["workload"] = describe(name, rr) + (" + MLP mobility correction" if mlp else "")
        extra[name + ("+mlp" if mlp else "")] = {k: (round(v, 4) if isinstance(v, float) else v)
                                                 for k, v in rr.items()}
        print("workload %s done" % name, file=sys.stderr, flush=True)
    return extra


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default 200 for the headline, else 5000)")
    ap.add_argument("--warmup", type=int, default=None, help="warm-up steps (default 20 for the headline, else 200)")
    ap.add_argument("--workload", default="headline", choices=["headline"] + sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--timing-steps", type=int, default=None,
                    help="eager steps timed per kernel launch (default 50 for the headline, else 500)")
    ap.add_argument("--all", action="store_true", help="also time the other workloads (reported under 'workloads')")
    ap.add_argument("--tune", action="store_true",
                    help="sweep tile x access variant on this workload and cache the fastest step under its name")
    ap.add_argument("--mlp", action="store_true",
                    help="colloid workloads: advance with the learned mobility correction (the MLP)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run 10 device copies of 512 MiB (reference for the HBM byte counters)")
    a = ap.parse_args()
    if a.copy_calibration:
        import torch
        src = torch.ones(1 << 27, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        from paper_0707_1299_amd import lbm
        for _ in range(10):
            dst.copy_(src)
        for _ in range(10):
            lbm.lb_copy_probe(src, dst)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each": 1 << 29, "copies": 10, "kernels": ["torch copy_", "lb_copy_probe"]}))
        return
    if a.tune:
        tune_workload(a.workload)
        return
    if a.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU decomposition "
              "(--gpus %d requested)" % a.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_0707_1299_amd import lbm  # noqa: F401  (fails loudly if the library is missing)

    hl = a.workload == "headline"
    a.steps = a.steps if a.steps is not None else (200 if hl else 5000)
    a.warmup = a.warmup if a.warmup is not None else (20 if hl else 200)
    a.timing_steps = a.timing_steps if a.timing_steps is not None else (50 if hl else 500)
    if hl:
        out = headline(a)
        if a.all:
            out["workloads"] = all_workloads()
        print(json.dumps(out))
        return
    if a.mlp and WORKLOADS[a.workload][3] not in ("colloids", "slab"):
        print("--mlp applies to the colloid workloads only", file=sys.stderr)
        sys.exit(2)
    r, inp = run_workload(a.workload, a.steps, a.warmup, a.timing_steps, mlp=a.mlp)
    same_bytes = BYTES_PER_NODE[inp[1]] * r["nodes"] // 2          # one population copy of the workload
    copy_gbs, copy_same_gbs = stream_copy_gbs(1 << 30), stream_copy_gbs(same_bytes)
    shape, storage, tau, kind, n, pos, frc, fkind, model = inp
    traffic = traffic_from_profile(a.workload, storage, r["nodes"])
    tile, variant = tuned(shape, storage, n if kind == "boxes" else 1, a.workload)
    out = {
        "metric": "MLUPS and % HBM roofline; colloid updates/s vs plain FP32 at stated error",
        "value": round(r["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(r["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp64": "f64", "fp16": "f16-storage/f32", "mom32": "f32"}[storage],
        "data": "synthetic",
        "config": {"workload": describe(a.workload, r) + (" + MLP mobility correction" if a.mlp else ""),
                   "nodes": r["nodes"], "points": r["points"],
                   "seed": 20261200 + {"singularities": 2, "colloids": 3, "slab": 3, "boxes": 4, "droplets": 5, "chains": 6}[kind],
                   "tile": list(tile or ()), "variant": variant},
        "roofline": {"bound": "hbm", "achieved": round(r["achieved_GBs"], 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(r["frac"], 4), "traffic": traffic,
                     "kernel": "k_lattice step (fused spread/pull/collide/store/interpolate)",
                     "bytes_per_node": BYTES_PER_NODE[storage], "kernel_ms": round(r["kernel_ms"], 5),
                     "launches_timed": r["launches_timed"],
                     "copy_1GiB_GBs": round(copy_gbs, 1), "frac_of_copy": round(r["achieved_GBs"] / copy_gbs, 4),
                     "copy_same_bytes_GBs": round(copy_same_gbs, 1),
                     "frac_of_copy_same_bytes": round(r["achieved_GBs"] / copy_same_gbs, 4)},
    }
    if "colloid_updates_per_s" in r:
        out["colloid_updates_per_s"] = round(r["colloid_updates_per_s"], 1)

    # (the CPU leg times the oracle's plain colloid update: none with --mlp)
    if not a.no_cpu and not a.mlp and kind in ("singularities", "colloids", "slab") and a.workload not in OPTS:
        box, csteps, cb = cpu_baseline(fkind, shape, storage, tau, pos, frc, model)
        out["cpu_baseline"] = cb
        # same number of steps on a fresh GPU lattice: error of this storage against the oracle
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            lat2, _ = build_lattice(shape, storage, tau, fkind, pos, frc, model, OPTS.get(a.workload))
            lat2.step(csteps)
            _, u = lat2.moments(rho=False)
            lat2.sync()
        _, uo = box.moments()
        err = float(np.abs(u.cpu().numpy()[0] - uo).max() / np.abs(uo).max())
        out["error_vs_oracle"] = {"velocity_rel_linf": err, "steps": csteps}

    if a.all:
        out["workloads"] = all_workloads()
        if not a.no_cpu:
            out["oracle_rates"] = oracle_rates()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
