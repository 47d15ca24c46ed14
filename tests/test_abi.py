"""The C-ABI library loads and exports every entry point include/lbm.h declares;
host-only calls (workspace sizing, argument checks, status strings and the
multipole helper) behave as documented.  No GPU work is launched here."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")

lbm = pytest.importorskip("paper_0707_1299_amd.lbm", reason="liblbm.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w \*]*?\b((?:lb|lbml)_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_documented_calls():
    names = declared_functions()
    for required in ("lb_init", "lb_add_point_forces", "lb_step", "lb_moments", "lb_interp_velocity",
                     "lb_workspace_bytes", "lb_diagnostics", "lb_sync", "lb_destroy", "lb_status_string",
                     "lb_last_error", "lbml_forward", "lbml_loss_grad", "lbml_adam_step", "lbml_loss_grad_static"):
        assert required in names


@pytest.mark.parametrize("name", declared_functions())
def test_symbol_exported(name):
    lib = ctypes.CDLL(lbm.LIB_PATH)
    assert hasattr(lib, name)
    out = subprocess.run(["nm", "-D", "--defined-only", lbm.LIB_PATH], capture_output=True, text=True).stdout
    assert re.search(r"\bT %s$" % name, out, flags=re.M)


def test_workspace_bytes_pure_and_monotone():
    a = lbm.lb_workspace_bytes(lbm.make_params((32, 32, 32), "fp32"))
    b = lbm.lb_workspace_bytes(lbm.make_params((32, 32, 32), "fp64"))
    c = lbm.lb_workspace_bytes(lbm.make_params((32, 32, 32), "fp16"))
    d = lbm.lb_workspace_bytes(lbm.make_params((32, 32, 32), "fp32", max_points=1000))
    assert c < a < b and d > a
    # two population copies of 19 planes dominate
    assert a >= 2 * 19 * 32 ** 3 * 4
    assert lbm.lb_workspace_bytes(lbm.make_params((32, 32, 32), "fp32")) == a
    # moment storage: two copies of 10 FP32 planes
    m = lbm.lb_workspace_bytes(lbm.make_params((32, 32, 32), "mom32"))
    assert 2 * 10 * 32 ** 3 * 4 <= m < a


@pytest.mark.parametrize("kw", [
    dict(shape=(3, 32, 32)), dict(shape=(32, 32, 2)), dict(nboxes=0), dict(storage=7),
    dict(max_points=-1), dict(tile=(64, 3, 1)), dict(variant=256), dict(variant=-1), dict(variant=132),
    dict(storage="mom32", tile=(16, 8, 2)), dict(collision=3), dict(collision=-1),
    dict(collision="mrt", ghost_rate=0.0), dict(collision="mrt", ghost_rate=4.5),
    dict(storage="mom32", collision="bgk"), dict(storage="mom32", collision="mrt", ghost_rate=1.5),
    dict(kT=-1e-5), dict(kT=float("inf")), dict(storage="mom32", kT=1e-5),
    dict(storage="fp16", fp16_exponent=121), dict(storage="fp16", fp16_exponent=-101),
    # boxes of 4 GiB or more need at least 64 lanes along x (box-relative offsets are 32-bit)
    dict(shape=(512, 512, 512), storage="fp32", tile=(32, 4, 2)),
    dict(shape=(512, 512, 512), storage="fp16", tile=(64, 2, 2)),     # two nodes per lane: 32 lanes
    dict(shape=(512, 512, 512), storage="fp16", tile=(32, 4, 2), variant=32),
])
def test_bad_params_rejected(kw):
    args = dict(shape=(16, 16, 16), storage="fp32")
    args.update(kw)
    p = lbm.make_params(**args)
    with pytest.raises(lbm.LBError) as e:
        lbm.lb_workspace_bytes(p)
    assert e.value.status in (lbm.LB_ERR_ARG, lbm.LB_ERR_SIZE)


def test_point_capacity_limits():
    """List entries pack the point index in 24 bits: 2^24 - 1 points are accepted, 2^24 are
    refused at set-up (with at most 64 tiles per point the entry count stays below 2^31)."""
    ok = lbm.lb_workspace_bytes(lbm.make_params((16, 16, 256), "fp32", max_points=(1 << 24) - 1, tile=(32, 4, 2)))
    assert ok > 0
    with pytest.raises(lbm.LBError) as e:
        lbm.lb_workspace_bytes(lbm.make_params((16, 16, 256), "fp32", max_points=1 << 24, tile=(32, 4, 2)))
    assert e.value.status == lbm.LB_ERR_SIZE


def test_status_strings():
    for code in (lbm.LB_OK, lbm.LB_ERR_ARG, lbm.LB_ERR_SIZE, lbm.LB_ERR_HIP, lbm.LB_ERR_NONFINITE,
                 lbm.LB_ERR_CAPACITY, lbm.LB_ERR_STATE, lbm.LB_ERR_NEGATIVE_DENSITY):
        s = lbm.lb_status_string(code)
        assert s and s != "unknown status"
    assert lbm.lb_status_string(12345) == "unknown status"


def test_expand_multipoles_matches_oracle():
    from oracle import multipole
    from paper_0707_1299_amd import workloads
    w = workloads.singularities(L=64, n=40)
    pos, frc = lbm.lb_expand_multipoles(w["types"], w["centers"], w["axes"], w["e1"], w["strengths"], w["sep"])
    opos, ofrc = multipole.expand(w["types"], w["centers"], w["axes"], w["e1"], w["strengths"], w["sep"])
    assert pos.shape == opos.shape
    assert np.abs(pos - opos).max() < 1e-13
    assert np.abs(frc - ofrc).max() < 1e-20


def test_expand_multipoles_rejects_unknown_type():
    with pytest.raises(lbm.LBError):
        lbm.lb_expand_multipoles([5], np.zeros((1, 3)), np.ones((1, 3)), np.ones((1, 3)), [1.0], 2.0)


def test_binding_fails_loudly_without_the_library():
    """No CPU fallback: importing the binding with the library absent raises ImportError."""
    import subprocess
    import sys
    code = (
        "import os, sys\n"
        "real = os.path.exists\n"
        "os.path.exists = lambda p: False if str(p).endswith('liblbm.so') else real(p)\n"
        "try:\n"
        "    import paper_0707_1299_amd.lbm\n"
        "except ImportError as e:\n"
        "    print('IMPORT_ERROR', e)\n"
        "    sys.exit(0)\n"
        "sys.exit(3)\n")
    root = __import__("os").path.dirname(__import__("os").path.dirname(__import__("os").path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "IMPORT_ERROR" in r.stdout


def test_copy_probe_rejects_bad_arguments_before_any_launch():
    """Argument checks of the streaming-copy probe run on the host: nothing is launched."""
    lib = lbm._L
    bad = [(0, 1 << 20, 64), (1 << 20, 0, 64), (1 << 20, 1 << 21, 0), (1 << 20, 1 << 21, 24),
           (1 << 20 | 8, 1 << 21, 64), (1 << 20, (1 << 21) | 4, 64), (1 << 20, (1 << 20) + 32, 64),
           ((1 << 20) + 32, 1 << 20, 64)]
    for s, d, n in bad:
        assert lib.lb_copy_probe(ctypes.c_void_p(s), ctypes.c_void_p(d), n, None) == lbm.LB_ERR_ARG, (s, d, n)


@pytest.mark.parametrize("shape,storage,tile,variant", [
    ((512, 512, 512), "fp16", (128, 2, 1), 0), ((512, 512, 512), "fp16", (64, 2, 2), 32),
    ((512, 512, 512), "fp32", (64, 4, 1), 0), ((512, 512, 512), "fp16", None, 0), ((512, 512, 512), "fp32", None, 0),
    ((256, 256, 256), "fp16", (64, 2, 2), 0)])
def test_big_box_tiles_accepted(shape, storage, tile, variant):
    """Whole-wave tile rows are accepted for boxes over 4 GiB (and the default tile is one)."""
    assert lbm.lb_workspace_bytes(lbm.make_params(shape, storage, tile=tile, variant=variant)) > 0


def test_tuned_entries_are_accepted_by_the_library():
    """Every (tile, variant) in the shipped tuning cache passes the library's own parameter
    checks for its storage and box shape (variant range, bit 128 only with one tile per block,
    tile shapes, whole-wave rows for large boxes), so no tuned workload is refused at set-up."""
    import json
    from paper_0707_1299_amd import tune
    cache = json.load(open(tune.CACHE))
    assert cache
    for key, e in cache.items():
        _, storage, dims, boxes = key.split("/")[:4]
        nx, ny, nz = map(int, dims.split("x"))
        v = int(e["variant"])
        assert 0 <= v <= 255 and not (v & 128 and (v >> 2) & 3), key
        p = lbm.make_params((nz, ny, nx), storage, nboxes=int(boxes[1:]), tile=tuple(e["tile"]), variant=v)
        assert lbm.lb_workspace_bytes(p) > 0, key
