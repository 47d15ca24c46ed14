"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU).

* The C oracle (oracle/lbm_oracle.c), built with gcc and the sanitizers,
  runs full steps on small non-cubic grids with points on and beyond the
  periodic seams (tests/asan_oracle_driver.c).
* The library's host code: every .hip source compiled with the sanitizers on
  the host pass (the device pass unoptimised and unsanitised), linked with
  tests/asan_host_driver.cpp, which drives the plan and workspace sizing over a
  grid of valid and invalid parameters, the argument checks of the entry
  points, the multipole expansion and the status strings.  Nothing touches a
  device.

Leak detection is off (the HIP runtime keeps its own allocations to the end);
any memory or undefined-behaviour error aborts the driver and fails the test.
"""
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests")
CSRC = os.path.join(ROOT, "paper_0707_1299_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, "%s\n%s\n%s" % (" ".join(cmd), r.stdout[-3000:], r.stderr[-3000:])
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_asan")
    _run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-ffp-contract=off",
          "-fopenmp", "-o", exe, os.path.join(HERE, "asan_oracle_driver.c"), os.path.join(ROOT, "oracle", "lbm_oracle.c"),
          "-lm"])
    r = _run([exe], env=dict(ENV, OMP_NUM_THREADS="2"), timeout=300)
    assert "oracle checks passed" in r.stdout


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_library_host_code_under_sanitizers(tmp_path):
    objs = []
    procs = []
    for src in sorted(glob.glob(os.path.join(CSRC, "*.hip"))):
        obj = str(tmp_path / (os.path.basename(src)[:-4] + ".o"))
        # each sanitizer flag applies to the host compilation alone (the device code is built
        # unoptimised, only so that the objects link; it never runs here)
        cmd = [HIPCC, "-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-fno-omit-frame-pointer", "-Xarch_device",
               "-O0", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-c", src, "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
        objs.append(obj)
    for cmd, p in procs:
        out, err = p.communicate(timeout=600)
        assert p.returncode == 0, "%s\n%s" % (" ".join(cmd), err[-3000:])
    drv = str(tmp_path / "driver.o")
    _run([HIPCC, "-x", "c++", "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer", "-Xarch_host", "-fsanitize=address",
          "-Xarch_host", "-fsanitize=undefined", "-c", os.path.join(HERE, "asan_host_driver.cpp"), "-o", drv],
         timeout=600)
    exe = str(tmp_path / "host_asan")
    _run([HIPCC, "-g", "-fno-omit-frame-pointer", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
          "-fsanitize=undefined", "-o", exe, drv] + objs, timeout=600)
    r = _run([exe], env=ENV, timeout=300)
    assert "host checks passed" in r.stdout
