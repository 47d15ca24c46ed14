"""FP64 CPU oracle for the forced MRT lattice Boltzmann step with point forces.

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg may import this package.  It shares no code
with the HIP library and imports nothing from it.

Layers (all FP64):
  * ``lbm_oracle.c``   plain C loops for spreading, collision, propagation,
                       interpolation and the colloid update (Secs. II-IV),
                       reached through ctypes below;
  * ``bruteforce``     the general scheme Eq. mrtlbe with an explicit 19x19
                       collision matrix, on tiny grids;
  * ``analytic``       closed forms: the exact DFT of the Peskin kernel, the
                       periodic Stokes / Oseen solution (Eq. oseen), the
                       Appendix A expression for a_L, the Hasimoto law;
  * ``multipole``      stresslet / rotlet expansion into point forces (Sec. III);
  * ``mlp``            the mobility-correction network in FP64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liblbm_oracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build_library(force: bool = False) -> str:
    """Compile the C oracle with gcc (no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build_library()
        L = ctypes.CDLL(_LIB)
        L.orc_phi.restype = ctypes.c_double
        L.orc_phi.argtypes = [ctypes.c_double]
        L.orc_velocities.argtypes = [_ip, _dp]
        L.orc_spread.argtypes = [ctypes.c_int] * 3 + [ctypes.c_int64, _dp, _dp, ctypes.c_int, _dp]
        L.orc_collide.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double, ctypes.c_double, _dp, _dp, _dp, _dp, _dp]
        L.orc_stream.argtypes = [ctypes.c_int] * 3 + [_dp, _dp]
        L.orc_moments.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double, _dp, _dp, _dp, _dp]
        L.orc_interp.argtypes = [ctypes.c_int] * 3 + [_dp, ctypes.c_int64, _dp, _dp]
        L.orc_advect.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double, ctypes.c_double, ctypes.c_int64,
                                                      _dp, _dp, _dp, _dp, _dp]
        L.orc_equilibrium.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double, _dp, _dp, _dp]
        L.orc_threads.restype = ctypes.c_int
        L.orc_threads.argtypes = []
        L.orc_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


def threads() -> int:
    """Threads the oracle's parallel loops use."""
    return lib().orc_threads()


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def phi(r: float) -> float:
    """Peskin's one-dimensional 4-point kernel, Eq. deltadef."""
    return lib().orc_phi(float(r))


def velocities():
    c = np.zeros((19, 3), dtype=np.int32)
    w = np.zeros(19, dtype=np.float64)
    lib().orc_velocities(c.ctypes.data_as(_ip), _p(w))
    return c.astype(np.int64), w


def spread(shape, pos, force, zero_net=False):
    """g(x) = sum_a F_a deltaP(x - R_a) (Sec. III); returns [3, nz, ny, nx]."""
    nz, ny, nx = shape
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    force = np.ascontiguousarray(force, dtype=np.float64).reshape(-1, 3)
    g = np.zeros((3, nz, ny, nx))
    lib().orc_spread(nx, ny, nz, len(pos), _p(pos), _p(force), int(bool(zero_net)), _p(g))
    return g


def collide(df, g, rho0, tau):
    """Projected-ghost MRT collision (Eq. fiexp); returns (df*, rho, u)."""
    _, nz, ny, nx = df.shape
    df = np.ascontiguousarray(df)
    out = np.empty_like(df)
    rho = np.empty((nz, ny, nx))
    u = np.empty((3, nz, ny, nx))
    gg = None if g is None else np.ascontiguousarray(g)
    lib().orc_collide(nx, ny, nz, rho0, tau, _p(df), _p(gg), _p(out), _p(rho), _p(u))
    return out, rho, u


def stream(dfstar):
    """df_i(x + c_i) = df*_i(x), periodic."""
    _, nz, ny, nx = dfstar.shape
    dfstar = np.ascontiguousarray(dfstar)
    out = np.empty_like(dfstar)
    lib().orc_stream(nx, ny, nz, _p(dfstar), _p(out))
    return out


def moments(df, g, rho0):
    """Physical rho and u = (sum fbar c + g/2)/rho (Eq. macrovariables2)."""
    _, nz, ny, nx = df.shape
    df = np.ascontiguousarray(df)
    rho = np.empty((nz, ny, nx))
    u = np.empty((3, nz, ny, nx))
    gg = None if g is None else np.ascontiguousarray(g)
    lib().orc_moments(nx, ny, nz, rho0, _p(df), _p(gg), _p(rho), _p(u))
    return rho, u


def interp(u, pos):
    """U(R) = sum_x u(x) deltaP(x - R) (Sec. IV)."""
    _, nz, ny, nx = u.shape
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    U = np.empty_like(pos)
    lib().orc_interp(nx, ny, nz, _p(np.ascontiguousarray(u)), len(pos), _p(pos), _p(U))
    return U


def advect(shape, rho0, tau, pos, force, U, inv_a, inv_aL):
    """R <- R + U + F/(6 pi eta)(1/a - 1/a_L), wrapped (Sec. IV).  Returns new positions."""
    nz, ny, nx = shape
    pos = np.array(pos, dtype=np.float64).reshape(-1, 3)
    n = len(pos)
    force = np.ascontiguousarray(force, dtype=np.float64).reshape(-1, 3)
    U = np.ascontiguousarray(U, dtype=np.float64).reshape(-1, 3)
    inv_a = np.ascontiguousarray(np.broadcast_to(np.asarray(inv_a, dtype=np.float64), (n,)))
    inv_aL = np.ascontiguousarray(np.broadcast_to(np.asarray(inv_aL, dtype=np.float64), (n,)))
    lib().orc_advect(nx, ny, nz, rho0, tau, n, _p(pos), _p(force), _p(U), _p(inv_a), _p(inv_aL))
    return pos


def equilibrium(rho, u, rho0):
    """Deviation of the Eq. eqf equilibrium from w_i rho0."""
    nz, ny, nx = rho.shape
    df = np.empty((19, nz, ny, nx))
    lib().orc_equilibrium(nx, ny, nz, rho0, _p(np.ascontiguousarray(rho, dtype=np.float64)),
                          _p(np.ascontiguousarray(u, dtype=np.float64)), _p(df))
    return df


@dataclass
class ForceSet:
    """Point forces for a run: ``kind`` is 'static' (fixed) or 'colloid' (advected)."""

    pos: np.ndarray
    force: np.ndarray
    kind: str = "static"
    inv_a: float | np.ndarray = 0.0
    inv_aL: float | np.ndarray = 0.0
    U: np.ndarray | None = None      # interpolated velocity of the last step
    inv_aL_fn: object = None         # optional callable(pos, tau) -> 1/a_L per particle


@dataclass
class Box:
    """A periodic box stepped by the oracle: state df is the pre-collision deviation."""

    shape: tuple
    tau: float
    rho0: float = 1.0
    zero_net_force: bool = False
    sets: list = field(default_factory=list)
    df: np.ndarray | None = None
    steps: int = 0

    def __post_init__(self):
        if self.df is None:
            self.df = np.zeros((19,) + tuple(self.shape))

    def _all_forces(self):
        if not self.sets:
            return np.zeros((0, 3)), np.zeros((0, 3))
        pos = np.concatenate([s.pos.reshape(-1, 3) for s in self.sets])
        frc = np.concatenate([s.force.reshape(-1, 3) for s in self.sets])
        return pos, frc

    def force_field(self):
        pos, frc = self._all_forces()
        return spread(self.shape, pos, frc, self.zero_net_force)

    def step(self, n: int = 1):
        """n steps of: spread -> moments -> interpolate -> collide -> propagate -> advance."""
        for _ in range(n):
            g = self.force_field()
            dfs, rho, u = collide(self.df, g, self.rho0, self.tau)
            for s in self.sets:
                s.U = interp(u, s.pos)
            self.df = stream(dfs)
            for s in self.sets:
                if s.kind == "colloid":
                    inv_aL = s.inv_aL if s.inv_aL_fn is None else s.inv_aL_fn(s.pos, self.tau)
                    s.pos = advect(self.shape, self.rho0, self.tau, s.pos, s.force, s.U, s.inv_a, inv_aL)
            self.steps += 1

    def moments(self):
        """Physical (rho, u) at the current time with the registered forces."""
        return moments(self.df, self.force_field(), self.rho0)

    def interp_velocity(self, pos):
        _, u = self.moments()
        return interp(u, pos)
