"""Closed-form references used to pin the oracle (TEST INFRASTRUCTURE ONLY).

* ``peskin_dft``      exact discrete Fourier transform of the spread kernel
                      deltaP(x - R) on a periodic lattice (Sec. III).
* ``oseen_modes``     the Stokes initial-value solution in Fourier space,
                      Eq. oseen: v(k,t) = (1 - exp(-eta k^2 t))/(eta k^2) (1 - kk).F(k).
* ``stokes_periodic`` its t -> infinity limit for a given force field, evaluated
                      by FFT (the periodic Hasimoto flow of the same spread force).
* ``inv_aL_appendix`` the Appendix A expression for 1/a_L (zz component).
* ``hasimoto``        v/v0 = 1/(1 + k a/L) with k = 2.84 (Fig. 5 caption).
* ``deltaapprox_ft``  Eq. deltaFT for the cosine approximation, Eq. deltaapprox.
"""
from __future__ import annotations

import numpy as np

from .bruteforce import peskin_1d


def kvectors(shape):
    """Angular wavenumbers k = 2 pi n / L on the lattice, each of shape (nz, ny, nx)."""
    nz, ny, nx = shape
    kz = 2 * np.pi * np.fft.fftfreq(nz)
    ky = 2 * np.pi * np.fft.fftfreq(ny)
    kx = 2 * np.pi * np.fft.fftfreq(nx)
    KZ, KY, KX = np.meshgrid(kz, ky, kx, indexing="ij")
    return KX, KY, KZ


def peskin_dft_1d(L, Rc):
    """sum_j phi(x_j - R) exp(-i k x_j) over the four support nodes, for k = 2 pi n / L."""
    k = 2 * np.pi * np.fft.fftfreq(L)
    base = int(np.floor(Rc))
    out = np.zeros(L, dtype=np.complex128)
    for xj in range(base - 1, base + 3):
        out += peskin_1d(xj - Rc) * np.exp(-1j * k * xj)
    return out


def peskin_dft(shape, R):
    """deltaP^(k; R) = prod_alpha of the one-dimensional transforms (numpy fftn convention)."""
    nz, ny, nx = shape
    fx = peskin_dft_1d(nx, R[0])
    fy = peskin_dft_1d(ny, R[1])
    fz = peskin_dft_1d(nz, R[2])
    return fz[:, None, None] * fy[None, :, None] * fx[None, None, :]


def transverse_project(KX, KY, KZ, Fk):
    """(1 - k^ k^) . F(k), Fk of shape (3, nz, ny, nx); the k = 0 mode is left unchanged."""
    k2 = KX ** 2 + KY ** 2 + KZ ** 2
    safe = np.where(k2 == 0, 1.0, k2)
    kdotF = (KX * Fk[0] + KY * Fk[1] + KZ * Fk[2]) / safe
    out = np.stack([Fk[0] - KX * kdotF, Fk[1] - KY * kdotF, Fk[2] - KZ * kdotF])
    return out, k2


def oseen_modes(g, eta, t):
    """Eq. oseen for a force field g (3, nz, ny, nx): returns v(k, t) for k != 0 (k = 0 set to 0)."""
    KX, KY, KZ = kvectors(g.shape[1:])
    Fk = np.fft.fftn(g, axes=(1, 2, 3))
    P, k2 = transverse_project(KX, KY, KZ, Fk)
    safe = np.where(k2 == 0, 1.0, k2)
    fac = np.where(k2 == 0, 0.0, (1 - np.exp(-eta * k2 * t)) / (eta * safe))
    return P * fac[None]


def stokes_periodic(g, eta):
    """Steady periodic Stokes flow of force field g (zero mean flow): ifft( P ghat / (eta k^2) )."""
    KX, KY, KZ = kvectors(g.shape[1:])
    Fk = np.fft.fftn(g, axes=(1, 2, 3))
    P, k2 = transverse_project(KX, KY, KZ, Fk)
    safe = np.where(k2 == 0, 1.0, k2)
    vk = np.where(k2[None] == 0, 0.0, P / (eta * safe[None]))
    return np.real(np.fft.ifftn(vk, axes=(1, 2, 3)))


def inv_aL_appendix(L, R, component=2):
    """Appendix A: 1/a_L = (6 pi / L^3) sum_{k != 0} |deltaP(k;R)|^2 / k^2 (1 - k^ k^)_cc,
    summed over the L^3 - 1 lattice wavevectors."""
    shape = (L, L, L)
    d = peskin_dft(shape, R)
    KX, KY, KZ = kvectors(shape)
    k2 = KX ** 2 + KY ** 2 + KZ ** 2
    kc = (KX, KY, KZ)[component]
    safe = np.where(k2 == 0, 1.0, k2)
    term = np.where(k2 == 0, 0.0, np.abs(d) ** 2 / safe * (1 - kc ** 2 / safe))
    return 6 * np.pi / L ** 3 * term.sum()


HASIMOTO_K = 2.84  # Fig. 5 caption


def hasimoto(a, L, k=HASIMOTO_K):
    """Steady sedimentation of a simple-cubic array: v / v0 = 1 / (1 + k a / L)."""
    return 1.0 / (1.0 + k * a / L)


def deltaapprox(r):
    """Eq. deltaapprox: (1 + cos(pi r / 2)) / 4 on |r| <= 2."""
    r = np.asarray(r, dtype=np.float64)
    return np.where(np.abs(r) <= 2, 0.25 * (1 + np.cos(np.pi * r / 2)), 0.0)


def deltaapprox_ft(k):
    """Eq. deltaFT, k in cycles: sinc(4 pi k) + sinc(4 pi k - pi)/2 + sinc(4 pi k + pi)/2,
    with sinc x = sin x / x."""
    def sinc(x):
        x = np.asarray(x, dtype=np.float64)
        return np.where(x == 0, 1.0, np.sin(x) / np.where(x == 0, 1.0, x))
    return sinc(4 * np.pi * k) + 0.5 * sinc(4 * np.pi * k - np.pi) + 0.5 * sinc(4 * np.pi * k + np.pi)
