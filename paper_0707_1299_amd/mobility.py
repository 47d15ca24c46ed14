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
3. ``evaluate``: on held-out single-particle runs, the error of the plain
   constant against the error of constant + MLP.

Host code here only arranges inputs and reads results; the lattice, the
interpolation and every network evaluation run in the HIP library.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

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
class Trained:
    master: object      # torch float32 [4545]
    w16: object         # torch int16 [4545] (bf16 bits)
    mu_plain: float
    out_scale: float
    losses: list

    def model(self, inv_a, **kw):
        return lbm.PointModel(inv_a=inv_a, inv_aL=self.mu_plain, mlp=self.w16, in_shift=IN_SHIFT, in_scale=IN_SCALE,
                              out_scale=self.out_scale, **kw)


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
    return Trained(master=master, w16=w16, mu_plain=float(mu_plain), out_scale=out_scale, losses=losses)


def predict(tr: Trained, offsets, taus):
    import torch
    x = torch.tensor(features(offsets, taus), device="cuda")
    y = torch.empty(len(x), dtype=torch.float32, device="cuda")
    lbm.lbml_forward(tr.w16, x, y)
    return tr.mu_plain + tr.out_scale * y.double().cpu().numpy()


def evaluate(tr: Trained, offsets, taus, mu_true):
    """RMS and max error of the plain constant and of constant + MLP against measured mu."""
    mu_true = np.asarray(mu_true, dtype=np.float64)
    pred = predict(tr, offsets, taus)
    e_plain = mu_true - tr.mu_plain
    e_mlp = mu_true - pred
    return dict(rms_plain=float(np.sqrt(np.mean(e_plain ** 2))), rms_mlp=float(np.sqrt(np.mean(e_mlp ** 2))),
                max_plain=float(np.abs(e_plain).max()), max_mlp=float(np.abs(e_mlp).max()),
                mu_mean=float(mu_true.mean()))
