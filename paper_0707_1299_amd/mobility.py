"""Learned correction to the lattice self-mobility 1/a_L (Sec. IV, Appendix A).

Workflow, all on the GPU through the C ABI:

1. ``single_particle_labels``: many independent 32^3 boxes in one batched
   context, one fixed colloid per box at a chosen sub-node offset and the
   box's own tau, counter-force on; the interpolated fluid velocity U is
   averaged over the last steps and turned into the dimensionless mobility
   mu(L) = 6 pi eta U.F / |F|^2 (1/a_L of Sec. IV at that offset, tau and box
   size L).  ``self_part`` removes the periodic images to first order,
   mu_self = mu(L) + k / L with the cubic-array coefficient k = 2.84 of the
   Fig. 5 law v = v0 / (1 + k a / L); mu_self is what the colloid update
   needs as 1/a_L so that a colloid in any box keeps the physical periodic
   slowdown.
2. ``train``: full-batch Adam on the library's MLP kernels (lbml_*), target
   (mu_self - mu_plain) / out_scale, features (2 o - 1, (tau - 1.05) / 0.45).
3. ``evaluate``: on held-out single-particle runs, the error of constant +
   MLP against two plain baselines: one constant for every tau, and the
   plain method of Sec. IV as it is used in practice, a_L fitted once for the
   run's own parameters, i.e. the offset-averaged label at the run's tau
   (``PlainTau``, a cubic fit in tau of the offset-averaged labels).
4. ``save`` / ``load``: a trained network as JSON (bf16 weights, input and
   output scaling, the plain baselines, training and held-out figures);
   ``python -m paper_0707_1299_amd.mobility --out FILE`` writes the network
   the benchmark and the full-size tests use.

Host code here only arranges inputs and reads results; the lattice, the
interpolation and every network evaluation run in the HIP library.
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import dataclass, field

import numpy as np

from . import lbm

IN_SHIFT = (0.5, 0.5, 0.5, 1.05)
IN_SCALE = (2.0, 2.0, 2.0, 1.0 / 0.45)
PERIODIC_K = 2.84   # v = v0 / (1 + k a / L) for a simple-cubic array (Fig. 5)


def self_part(mu, L):
    """Lattice self-mobility with the periodic images removed to first order."""
    return np.asarray(mu, dtype=np.float64) + PERIODIC_K / L


def features(offsets, taus):
    o = np.asarray(offsets, dtype=np.float64)
    t = np.asarray(taus, dtype=np.float64)
    x = np.empty((len(o), 4), dtype=np.float32)
    for k in range(3):
        x[:, k] = (o[:, k] - IN_SHIFT[k]) * IN_SCALE[k]
    x[:, 3] = (t - IN_SHIFT[3]) * IN_SCALE[3]
    return x


def single_particle_labels(offsets, taus, L=32, steps=2000, average=200, fz=-1e-6, storage="fp32", rho0=1.0):
    """One colloid per box at (L/2, L/2, L/2) + offset; returns mu per box (FP64 numpy)."""
    import torch
    offsets = np.asarray(offsets, dtype=np.float64)
    taus = np.asarray(taus, dtype=np.float64)
    n = len(offsets)
    pos = np.full((n, 3), L / 2.0) + offsets
    frc = np.tile([0.0, 0.0, fz], (n, 1))
    lat = lbm.Lattice((L, L, L), storage, nboxes=n, tau=taus, rho0=rho0, zero_net_force=True, max_points=n)
    dpos = torch.tensor(pos, dtype=torch.float64, device="cuda")
    dfrc = torch.tensor(frc, dtype=torch.float64, device="cuda")
    dbox = torch.arange(n, dtype=torch.int32, device="cuda")
    vsum = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
    lat.add_point_forces(dpos, dfrc, dbox, lbm.LB_FORCES_STATIC, lbm.PointModel(vel_sum=vsum))
    lat.step(steps - average)
    vsum.zero_()
    lat.step(average)
    lat.sync()
    U = vsum.cpu().numpy() / average
    eta = rho0 * taus / 3.0
    mu = 6 * math.pi * eta * U[:, 2] / fz
    lat.close()
    return mu


@dataclass
class PlainTau:
    """The plain method's a_L for a run at a given tau: the offset average of the labels,
    fitted as a cubic in tau by least squares over the training labels."""
    coef: list          # numpy.polyfit order (highest power first)
    tau_range: tuple

    @classmethod
    def fit(cls, taus, mu, deg=3):
        taus = np.asarray(taus, dtype=np.float64)
        return cls(coef=[float(c) for c in np.polyfit(taus, np.asarray(mu, dtype=np.float64), deg)],
                   tau_range=(float(taus.min()), float(taus.max())))

    def __call__(self, taus):
        return np.polyval(np.asarray(self.coef), np.asarray(taus, dtype=np.float64))


@dataclass
class Trained:
    master: object      # torch float32 [4545] (None for a loaded network)
    w16: object         # torch int16 [4545] (bf16 bits)
    mu_plain: float
    out_scale: float
    losses: list
    plain_tau: PlainTau | None = None
    meta: dict = field(default_factory=dict)

    def model(self, inv_a, **kw):
        return lbm.PointModel(inv_a=inv_a, inv_aL=self.mu_plain, mlp=self.w16, in_shift=IN_SHIFT, in_scale=IN_SCALE,
                              out_scale=self.out_scale, **kw)

    def plain_model(self, inv_a, tau, **kw):
        """The plain method for a run at this tau: the constant 1/a_L fitted for it, no network."""
        return lbm.PointModel(inv_a=inv_a, inv_aL=float(self.plain_tau(tau)), **kw)


def init_master(seed=0):
    """Glorot-uniform weights, zero biases (float32), in the lbml layout."""
    rng = np.random.default_rng(seed)
    parts = []
    for shape in ((64, 4), (64,), (64, 64), (64,), (1, 64), (1,)):
        if len(shape) == 2:
            lim = math.sqrt(6.0 / (shape[0] + shape[1]))
            parts.append(rng.uniform(-lim, lim, size=shape).ravel())
        else:
            parts.append(np.zeros(shape))
    return np.concatenate(parts).astype(np.float32)


def train(offsets, taus, mu, mu_plain=None, iters=3000, lr=3e-3, seed=0):
    import torch
    mu = np.asarray(mu, dtype=np.float64)
    if mu_plain is None:
        mu_plain = float(mu.mean())
    resid = mu - mu_plain
    out_scale = float(max(np.abs(resid).max(), 1e-12))
    x = torch.tensor(features(offsets, taus), device="cuda")
    y = torch.tensor((resid / out_scale).astype(np.float32), device="cuda")
    n = len(mu)
    master = torch.tensor(init_master(seed), device="cuda")
    m = torch.zeros_like(master)
    v = torch.zeros_like(master)
    grad = torch.zeros_like(master)
    w16 = torch.zeros(lbm.LBML_NPARAM, dtype=torch.int16, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    work = torch.empty(lbm.lbml_work_floats(n), dtype=torch.float32, device="cuda")
    lbm.lbml_round_bf16(master, w16)
    losses = []
    for t in range(1, iters + 1):
        lbm.lbml_loss_grad(w16, x, y, grad, loss, work)
        lbm.lbml_adam_step(master, m, v, grad, w16, t, lr=lr)
        if t == 1 or t % 100 == 0:
            losses.append((t, float(loss.item())))
    return Trained(master=master, w16=w16, mu_plain=float(mu_plain), out_scale=out_scale, losses=losses,
                   plain_tau=PlainTau.fit(taus, mu))


def predict(tr: Trained, offsets, taus):
    import torch
    x = torch.tensor(features(offsets, taus), device="cuda")
    y = torch.empty(len(x), dtype=torch.float32, device="cuda")
    lbm.lbml_forward(tr.w16, x, y)
    return tr.mu_plain + tr.out_scale * y.double().cpu().numpy()


def evaluate(tr: Trained, offsets, taus, mu_true):
    """RMS and max error against measured mu of: the one constant for every tau (plain), the
    offset-averaged constant fitted for each run's tau (plain_tau, the plain method of Sec. IV),
    and constant + MLP (mlp)."""
    mu_true = np.asarray(mu_true, dtype=np.float64)
    pred = predict(tr, offsets, taus)
    errs = dict(plain=mu_true - tr.mu_plain, mlp=mu_true - pred)
    if tr.plain_tau is not None:
        errs["plain_tau"] = mu_true - tr.plain_tau(taus)
    out = dict(mu_mean=float(mu_true.mean()), n=int(len(mu_true)))
    for k, e in errs.items():
        out["rms_" + k] = float(np.sqrt(np.mean(e ** 2)))
        out["max_" + k] = float(np.abs(e).max())
    return out


def save(tr: Trained, path, **meta):
    """Write a trained network (bf16 weights as 16-bit integers) and its baselines as JSON."""
    w = tr.w16.cpu().numpy().astype(np.int64) & 0xFFFF
    d = dict(format="lbml-4-64-64-1-bf16", nparam=lbm.LBML_NPARAM, w16=[int(v) for v in w],
             in_shift=list(IN_SHIFT), in_scale=list(IN_SCALE), out_scale=tr.out_scale, mu_plain=tr.mu_plain,
             plain_tau=None if tr.plain_tau is None else dict(coef=tr.plain_tau.coef,
                                                              tau_range=list(tr.plain_tau.tau_range)),
             losses=tr.losses, meta=dict(tr.meta, **meta))
    with open(path, "w") as f:
        json.dump(d, f, indent=1)


def load(path):
    """A network written by save(), its weights on the current device."""
    import torch
    with open(path) as f:
        d = json.load(f)
    if d.get("format") != "lbml-4-64-64-1-bf16" or d.get("nparam") != lbm.LBML_NPARAM:
        raise ValueError("%s: not a 4-64-64-1 bf16 mobility network" % path)
    if tuple(d["in_shift"]) != IN_SHIFT or tuple(d["in_scale"]) != IN_SCALE:
        raise ValueError("%s: input scaling differs from this module's" % path)
    w = np.asarray(d["w16"], dtype=np.uint16).view(np.int16)
    w16 = torch.tensor(w, dtype=torch.int16, device="cuda")
    pt = d.get("plain_tau")
    return Trained(master=None, w16=w16, mu_plain=float(d["mu_plain"]), out_scale=float(d["out_scale"]),
                   losses=d.get("losses", []),
                   plain_tau=None if pt is None else PlainTau(coef=pt["coef"], tau_range=tuple(pt["tau_range"])),
                   meta=d.get("meta", {}))


def weights_f64(tr: Trained):
    """The network's bf16 weights as FP64 values (host), in the lbml layout."""
    b = tr.w16.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)


DEFAULT_NET = os.path.join(os.path.dirname(os.path.abspath(__file__)), "mobility_net.json")


def main(argv=None):
    """Label generation, training and held-out evaluation of the network that the benchmark and
    the full-size tests load: single-particle 32^3 boxes generated by the batched library,
    tau ~ U[0.5, 1.5] (the batched workload's range widened down to the tau = 1/2 of the large
    colloid workloads), offsets ~ U[0, 1)^3; every step on the GPU."""
    import argparse
    import time
    from . import workloads
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_NET)
    ap.add_argument("--train", type=int, default=1024)
    ap.add_argument("--test", type=int, default=256)
    ap.add_argument("--test-half", type=int, default=128, help="held-out runs at tau = 1/2")
    ap.add_argument("--iters", type=int, default=6000)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--L", type=int, default=32)
    a = ap.parse_args(argv)
    t0 = time.time()
    g = workloads.rng(7)
    tau_lo, tau_hi = 0.5, 1.5
    off_tr = g.uniform(0, 1, size=(a.train, 3))
    tau_tr = g.uniform(tau_lo, tau_hi, size=a.train)
    off_te = g.uniform(0, 1, size=(a.test, 3))
    tau_te = g.uniform(tau_lo, tau_hi, size=a.test)
    off_h = g.uniform(0, 1, size=(a.test_half, 3))
    tau_h = np.full(a.test_half, 0.5)
    lab = dict(L=a.L, steps=2000, average=200)
    mu_tr = self_part(single_particle_labels(off_tr, tau_tr, **lab), a.L)
    mu_te = self_part(single_particle_labels(off_te, tau_te, **lab), a.L)
    mu_h = self_part(single_particle_labels(off_h, tau_h, **lab), a.L)
    print("labels: %d + %d + %d runs, %.1f s" % (a.train, a.test, a.test_half, time.time() - t0), flush=True)
    tr = train(off_tr, tau_tr, mu_tr, iters=a.iters, lr=a.lr)
    print("trained: loss %.3e -> %.3e, %.1f s" % (tr.losses[0][1], tr.losses[-1][1], time.time() - t0), flush=True)
    ev = evaluate(tr, off_te, tau_te, mu_te)
    evh = evaluate(tr, off_h, tau_h, mu_h)
    print("held-out (tau ~ U[%.1f, %.1f]): %s" % (tau_lo, tau_hi, json.dumps(ev)), flush=True)
    print("held-out (tau = 1/2): %s" % json.dumps(evh), flush=True)
    save(tr, a.out, labels=dict(L=a.L, steps=2000, average=200, fz=-1e-6, storage="fp32", seed_index=7,
                                n_train=a.train, tau_range=[tau_lo, tau_hi], target="mu(L) + 2.84/L"),
         training=dict(iters=a.iters, lr=a.lr, init_seed=0), held_out=ev, held_out_tau_half=evh)
    print("wrote %s" % a.out)


if __name__ == "__main__":
    main()
