"""ctypes binding of liblbm (include/lbm.h).

Argument marshalling only: every step of the method runs in the HIP library.
The functions keep the C names; ``Lattice`` is a convenience holder that
allocates the workspace as a torch uint8 tensor on the current device and
passes ``data_ptr()`` values and the current stream.  If the built library is
missing this module raises ImportError; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "liblbm.so")

LB_OK = 0
LB_ERR_ARG = -1
LB_ERR_SIZE = -2
LB_ERR_HIP = -3
LB_ERR_NONFINITE = -4
LB_ERR_CAPACITY = -5
LB_ERR_STATE = -6
LB_ERR_NEGATIVE_DENSITY = -7

LB_STORAGE_FP64 = 0
LB_STORAGE_FP32 = 1
LB_STORAGE_FP16 = 2
LB_STORAGE_MOM32 = 3

LB_COLLISION_PROJECTED = 0
LB_COLLISION_BGK = 1
LB_COLLISION_MRT = 2
COLLISION = {"projected": LB_COLLISION_PROJECTED, "bgk": LB_COLLISION_BGK, "mrt": LB_COLLISION_MRT}

LB_FORCES_NEXT_STEP = 0
LB_FORCES_STATIC = 1
LB_COLLOIDS = 2

LB_NDIAG = 13
LBML_NPARAM = 4545

STORAGE = {"fp64": LB_STORAGE_FP64, "fp32": LB_STORAGE_FP32, "fp16": LB_STORAGE_FP16, "mom32": LB_STORAGE_MOM32}


class lb_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("nboxes", ctypes.c_int32), ("storage", ctypes.c_int32), ("zero_net_force", ctypes.c_int32),
        ("rho0", ctypes.c_double), ("tau", ctypes.POINTER(ctypes.c_double)),
        ("max_points", ctypes.c_int64),
        ("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32), ("tile_z", ctypes.c_int32),
        ("fp16_exponent", ctypes.c_int32), ("variant", ctypes.c_int32),
        ("collision", ctypes.c_int32), ("tau_bulk", ctypes.POINTER(ctypes.c_double)),
        ("ghost_rate", ctypes.c_double), ("kT", ctypes.c_double), ("seed", ctypes.c_uint64),
    ]


class lb_point_model(ctypes.Structure):
    _fields_ = [
        ("inv_a", ctypes.c_double), ("inv_aL", ctypes.c_double),
        ("d_mlp", ctypes.c_void_p),
        ("in_shift", ctypes.c_float * 4), ("in_scale", ctypes.c_float * 4), ("out_scale", ctypes.c_float),
        ("d_vel_out", ctypes.c_void_p), ("d_vel_sum", ctypes.c_void_p),
    ]


LB_ELASTIC_CHAIN = 0
LB_ELASTIC_SURFACE = 1


class lb_elastic(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32), ("chain_len", ctypes.c_int32), ("n", ctypes.c_int64),
        ("d_pos", ctypes.c_void_p), ("d_force", ctypes.c_void_p), ("d_ext", ctypes.c_void_p),
        ("d_box", ctypes.c_void_p), ("d_vel_out", ctypes.c_void_p),
        ("k_spring", ctypes.c_double), ("l0", ctypes.c_double), ("tension", ctypes.c_double),
        ("ntri", ctypes.c_int64), ("d_tri", ctypes.c_void_p), ("d_vt_off", ctypes.c_void_p),
        ("d_vt_idx", ctypes.c_void_p),
    ]


def vertex_triangle_incidence(tri, nverts):
    """CSR lists of the triangles containing each vertex, ascending (host side)."""
    tri = np.asarray(tri, dtype=np.int64).reshape(-1, 3)
    t = np.repeat(np.arange(len(tri)), 3)
    v = tri.ravel()
    order = np.lexsort((t, v))
    counts = np.bincount(v, minlength=nverts)
    off = np.zeros(nverts + 1, dtype=np.int32)
    off[1:] = np.cumsum(counts)
    return off, t[order].astype(np.int32)


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("liblbm.so is not built (%s); run python -m paper_0707_1299_amd.build" % LIB_PATH)
    # torch ships its own HIP runtime under the same soname; load it first so
    # that the library binds to that one instead of a second runtime from
    # /opt/rocm (two runtimes in one process do not share the device).
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "lb_workspace_bytes": (ctypes.c_int, [P(lb_params), P(ctypes.c_size_t)]),
        "lb_init": (ctypes.c_int, [P(lb_params), vp, ctypes.c_size_t, vp, P(vp)]),
        "lb_set_stream": (ctypes.c_int, [vp, vp]),
        "lb_set_equilibrium": (ctypes.c_int, [vp, vp, vp]),
        "lb_add_point_forces": (ctypes.c_int, [vp, i64, vp, vp, vp, ctypes.c_int, P(lb_point_model)]),
        "lb_clear_forces": (ctypes.c_int, [vp]),
        "lb_add_elastic": (ctypes.c_int, [vp, P(lb_elastic)]),
        "lb_step": (ctypes.c_int, [vp, i32]),
        "lb_prepare_steps": (ctypes.c_int, [vp, i32]),
        "lb_moments": (ctypes.c_int, [vp, vp, vp]),
        "lb_interp_velocity": (ctypes.c_int, [vp, i64, vp, vp, vp]),
        "lb_diagnostics": (ctypes.c_int, [vp, P(dbl)]),
        "lb_sync": (ctypes.c_int, [vp]),
        "lb_destroy": (ctypes.c_int, [vp]),
        "lb_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "lb_last_error": (ctypes.c_char_p, [vp]),
        "lb_steps_taken": (i64, [vp]),
        "lb_checkpoint_bytes": (ctypes.c_int, [vp, P(ctypes.c_size_t)]),
        "lb_checkpoint_save": (ctypes.c_int, [vp, vp]),
        "lb_checkpoint_load": (ctypes.c_int, [vp, vp]),
        "lb_kernel_timing": (ctypes.c_int, [vp, ctypes.c_int]),
        "lb_kernel_time": (ctypes.c_int, [vp, P(dbl), P(i64)]),
        "lb_copy_probe": (ctypes.c_int, [vp, vp, ctypes.c_size_t, vp]),
        "lb_expand_multipoles": (ctypes.c_int, [i64, vp, vp, vp, vp, vp, dbl, P(i64), vp, vp]),
        "lbml_work_floats": (i64, [i64]),
        "lbml_round_bf16": (ctypes.c_int, [vp, vp, vp]),
        "lbml_forward": (ctypes.c_int, [vp, i64, vp, vp, vp]),
        "lbml_loss_grad": (ctypes.c_int, [vp, i64, vp, vp, vp, vp, vp, vp]),
        "lbml_loss_grad_static": (ctypes.c_int, [vp, i64, vp, vp, vp, vp, vp]),
        "lbml_adam_step": (ctypes.c_int, [vp, vp, vp, vp, vp, i32, ctypes.c_float, ctypes.c_float,
                                          ctypes.c_float, ctypes.c_float, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


_L = _load()


class LBError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        super().__init__("%s (%d)%s" % (lb_status_string(status), status, (": " + msg) if msg else ""))


def lb_status_string(status: int) -> str:
    return _L.lb_status_string(int(status)).decode()


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream_handle():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def make_params(shape, storage="fp32", nboxes=1, tau=0.5, rho0=1.0, zero_net_force=False, max_points=0,
                tile=None, fp16_exponent=0, variant=0, collision="projected", tau_bulk=None, ghost_rate=2.0, kT=0.0,
                seed=0):
    """lb_params for boxes of shape (nz, ny, nx); tau and tau_bulk are scalars or per-box sequences."""
    nz, ny, nx = shape
    taus = np.ascontiguousarray(np.broadcast_to(np.asarray(tau, dtype=np.float64), (nboxes,)))
    p = lb_params()
    p.nx, p.ny, p.nz = nx, ny, nz
    p.nboxes = nboxes
    p.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    p.zero_net_force = int(bool(zero_net_force))
    p.rho0 = rho0
    p.tau = taus.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    p.max_points = max_points
    if tile:
        p.tile_x, p.tile_y, p.tile_z = tile
    p.fp16_exponent = fp16_exponent
    p.variant = variant
    p.collision = COLLISION[collision] if isinstance(collision, str) else int(collision)
    p.ghost_rate = ghost_rate
    p.kT = kT
    p.seed = seed
    p._taus = taus  # keep alive
    if tau_bulk is not None:
        tb = np.ascontiguousarray(np.broadcast_to(np.asarray(tau_bulk, dtype=np.float64), (nboxes,)))
        p.tau_bulk = tb.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        p._tau_bulk = tb
    return p


def lb_workspace_bytes(p: lb_params) -> int:
    n = ctypes.c_size_t(0)
    r = _L.lb_workspace_bytes(ctypes.byref(p), ctypes.byref(n))
    if r != LB_OK:
        raise LBError(r, _L.lb_last_error(None).decode())
    return n.value


def lb_expand_multipoles(types, centers, axes, e1s, strengths, sep):
    """Host-side expansion of multipoles into point forces (see include/lbm.h)."""
    types = np.ascontiguousarray(types, dtype=np.int32)
    n = len(types)
    c = np.ascontiguousarray(centers, dtype=np.float64).reshape(n, 3)
    a = np.ascontiguousarray(axes, dtype=np.float64).reshape(n, 3)
    e = np.ascontiguousarray(e1s, dtype=np.float64).reshape(n, 3)
    s = np.ascontiguousarray(strengths, dtype=np.float64).reshape(n)
    pos = np.zeros((4 * n, 3))
    frc = np.zeros((4 * n, 3))
    m = ctypes.c_int64(0)
    r = _L.lb_expand_multipoles(n, types.ctypes.data, c.ctypes.data, a.ctypes.data, e.ctypes.data, s.ctypes.data,
                                float(sep), ctypes.byref(m), pos.ctypes.data, frc.ctypes.data)
    if r != LB_OK:
        raise LBError(r)
    return pos[:m.value].copy(), frc[:m.value].copy()


@dataclass
class PointModel:
    inv_a: float = 0.0
    inv_aL: float = 0.0
    mlp: object = None          # torch uint16/int16 tensor of LBML_NPARAM bf16 weights
    in_shift: tuple = (0.0, 0.0, 0.0, 0.0)
    in_scale: tuple = (1.0, 1.0, 1.0, 1.0)
    out_scale: float = 1.0
    vel_out: object = None      # torch float64 (n,3)
    vel_sum: object = None      # torch float64 (n,3)

    def to_c(self):
        m = lb_point_model()
        m.inv_a, m.inv_aL = self.inv_a, self.inv_aL
        m.d_mlp = None if self.mlp is None else self.mlp.data_ptr()
        for k in range(4):
            m.in_shift[k] = self.in_shift[k]
            m.in_scale[k] = self.in_scale[k]
        m.out_scale = self.out_scale
        m.d_vel_out = None if self.vel_out is None else self.vel_out.data_ptr()
        m.d_vel_sum = None if self.vel_sum is None else self.vel_sum.data_ptr()
        return m


class Lattice:
    """One liblbm context on the current torch device and stream."""

    def __init__(self, shape, storage="fp32", nboxes=1, tau=0.5, rho0=1.0, zero_net_force=False, max_points=0,
                 tile=None, fp16_exponent=0, variant=0, stream=None, collision="projected", tau_bulk=None,
                 ghost_rate=2.0, kT=0.0, seed=0):
        import torch
        self.torch = torch
        self.shape = tuple(shape)
        self.nboxes = nboxes
        self.params = make_params(shape, storage, nboxes, tau, rho0, zero_net_force, max_points, tile,
                                  fp16_exponent, variant, collision, tau_bulk, ghost_rate, kT, seed)
        nbytes = lb_workspace_bytes(self.params)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        base = self.workspace.data_ptr()
        self._ws = base + ((-base) % 256)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        ctx = ctypes.c_void_p()
        r = _L.lb_init(ctypes.byref(self.params), ctypes.c_void_p(self._ws), nbytes,
                       ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx))
        if r != LB_OK:
            raise LBError(r, _L.lb_last_error(None).decode())
        self.ctx = ctx
        self._keep = []   # tensors that must outlive their use by queued work

    def _check(self, r):
        if r != LB_OK:
            raise LBError(r, _L.lb_last_error(self.ctx).decode())

    def close(self):
        if getattr(self, "ctx", None):
            _L.lb_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_equilibrium(self, rho, u):
        self._check(_L.lb_set_equilibrium(self.ctx, _ptr(rho), _ptr(u)))
        self._keep += [rho, u]

    def add_point_forces(self, pos, force, box=None, kind=LB_FORCES_STATIC, model: PointModel | None = None):
        """pos, force: torch float64 (n,3) on the device; box: torch int32 (n) or None."""
        n = pos.shape[0]
        m = None if model is None else ctypes.byref(model.to_c())
        self._check(_L.lb_add_point_forces(self.ctx, n, _ptr(pos), _ptr(force), _ptr(box), kind, m))
        self._keep += [pos, force, box, model]

    def add_chains(self, pos, chain_len, k_spring, l0, ext=None, box=None, vel_out=None):
        """Bead-spring chains of chain_len consecutive markers; pos torch float64 (n,3), moved in place.
        Returns the (n,3) tensor the library writes the marker forces into."""
        e = lb_elastic()
        e.kind, e.chain_len, e.n = LB_ELASTIC_CHAIN, chain_len, pos.shape[0]
        e.k_spring, e.l0 = k_spring, l0
        return self._add_elastic(e, pos, ext, box, vel_out, [])

    def add_surface(self, pos, tri, tension, ext=None, box=None, vel_out=None):
        """Closed triangulated surface (tri (ntri,3), counter-clockwise about the outward normal) of
        the given tension; pos torch float64 (n,3), moved in place.  Returns the marker-force tensor."""
        t = self.torch
        tri_np = np.asarray(tri, dtype=np.int32).reshape(-1, 3)
        off, idx = vertex_triangle_incidence(tri_np, pos.shape[0])
        d_tri = t.tensor(tri_np, device="cuda")
        d_off = t.tensor(off, device="cuda")
        d_idx = t.tensor(idx, device="cuda")
        e = lb_elastic()
        e.kind, e.n, e.tension, e.ntri = LB_ELASTIC_SURFACE, pos.shape[0], tension, len(tri_np)
        e.d_tri, e.d_vt_off, e.d_vt_idx = _ptr(d_tri), _ptr(d_off), _ptr(d_idx)
        return self._add_elastic(e, pos, ext, box, vel_out, [d_tri, d_off, d_idx])

    def _add_elastic(self, e, pos, ext, box, vel_out, keep):
        frc = self.torch.zeros_like(pos)
        e.d_pos, e.d_force, e.d_ext, e.d_box, e.d_vel_out = _ptr(pos), _ptr(frc), _ptr(ext), _ptr(box), _ptr(vel_out)
        self._check(_L.lb_add_elastic(self.ctx, ctypes.byref(e)))
        self._keep += [pos, frc, ext, box, vel_out] + keep
        return frc

    def clear_forces(self):
        self._check(_L.lb_clear_forces(self.ctx))

    def step(self, n=1):
        self._check(_L.lb_step(self.ctx, n))

    def prepare_steps(self, n):
        """Capture the HIP graphs step(n) would replay, without taking a step."""
        self._check(_L.lb_prepare_steps(self.ctx, n))

    def moments(self, rho=True):
        t = self.torch
        nz, ny, nx = self.shape
        u = t.empty((self.nboxes, 3, nz, ny, nx), dtype=t.float64, device="cuda")
        r = t.empty((self.nboxes, nz, ny, nx), dtype=t.float64, device="cuda") if rho else None
        self._check(_L.lb_moments(self.ctx, _ptr(r), _ptr(u)))
        return r, u

    def interp_velocity(self, pos, box=None):
        t = self.torch
        out = t.empty((pos.shape[0], 3), dtype=t.float64, device="cuda")
        self._check(_L.lb_interp_velocity(self.ctx, pos.shape[0], _ptr(pos), _ptr(box), _ptr(out)))
        return out

    def diagnostics(self):
        out = np.zeros((self.nboxes, LB_NDIAG))
        r = _L.lb_diagnostics(self.ctx, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        return r, out

    def sync(self):
        self._check(_L.lb_sync(self.ctx))

    def steps_taken(self):
        return int(_L.lb_steps_taken(self.ctx))

    def checkpoint_bytes(self):
        n = ctypes.c_size_t(0)
        self._check(_L.lb_checkpoint_bytes(self.ctx, ctypes.byref(n)))
        return n.value

    def checkpoint_save(self, buf):
        """Copy the state into buf (a device uint8 tensor of at least checkpoint_bytes() + 256 bytes);
        returns the 256-byte aligned address used."""
        p = buf.data_ptr() + ((-buf.data_ptr()) % 256)
        self._check(_L.lb_checkpoint_save(self.ctx, ctypes.c_void_p(p)))
        return p

    def checkpoint_load(self, buf):
        p = buf.data_ptr() + ((-buf.data_ptr()) % 256)
        self._check(_L.lb_checkpoint_load(self.ctx, ctypes.c_void_p(p)))

    def kernel_timing(self, enable=True):
        self._check(_L.lb_kernel_timing(self.ctx, int(bool(enable))))

    def kernel_time(self):
        ms = ctypes.c_double(0)
        n = ctypes.c_int64(0)
        self._check(_L.lb_kernel_time(self.ctx, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value


# ---- MLP entry points -------------------------------------------------------

def lbml_work_floats(n):
    return int(_L.lbml_work_floats(n))


def lbml_round_bf16(master, w16):
    r = _L.lbml_round_bf16(_ptr(master), _ptr(w16), _stream_handle())
    if r != LB_OK:
        raise LBError(r)


def lbml_forward(w16, x, y):
    r = _L.lbml_forward(_ptr(w16), x.shape[0], _ptr(x), _ptr(y), _stream_handle())
    if r != LB_OK:
        raise LBError(r)


def lbml_loss_grad(w16, x, target, grad, loss, work):
    r = _L.lbml_loss_grad(_ptr(w16), x.shape[0], _ptr(x), _ptr(target), _ptr(grad), _ptr(loss), _ptr(work),
                          _stream_handle())
    if r != LB_OK:
        raise LBError(r)


LBML_STATIC_MAX_N = 4096


def lbml_loss_grad_static(w16, x, target, grad, loss):
    """lbml_loss_grad with the library's own work array (no work argument; n <= LBML_STATIC_MAX_N)."""
    r = _L.lbml_loss_grad_static(_ptr(w16), x.shape[0], _ptr(x), _ptr(target), _ptr(grad), _ptr(loss),
                                 _stream_handle())
    if r != LB_OK:
        raise LBError(r)


def lbml_adam_step(master, m, v, grad, w16, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    r = _L.lbml_adam_step(_ptr(master), _ptr(m), _ptr(v), _ptr(grad), _ptr(w16), int(t), lr, beta1, beta2, eps,
                          _stream_handle())
    if r != LB_OK:
        raise LBError(r)


def lb_copy_probe(src, dst, nbytes=None):
    """Streaming copy of nbytes (default: all of src) from src to dst, device tensors, on torch's current
    stream; a measurement aid for the HBM copy rate."""
    nbytes = src.numel() * src.element_size() if nbytes is None else int(nbytes)
    if nbytes > dst.numel() * dst.element_size() or nbytes > src.numel() * src.element_size():
        raise LBError(LB_ERR_ARG, "copy larger than a buffer")
    r = _L.lb_copy_probe(_ptr(src), _ptr(dst), nbytes, _stream_handle())
    if r != LB_OK:
        raise LBError(r)
