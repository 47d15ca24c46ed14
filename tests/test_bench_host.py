"""Host logic of bench.py (no GPU): the one-GPU refusal, the staleness rules of the
committed HBM-traffic record, and the two-pass workload tuner."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_mlp_only_for_colloid_workloads():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--mlp", "--workload", "singularities128"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "colloid" in r.stderr


def _record(tmp_path, monkeypatch, **over):
    """A traffic record for the default workload in a scratch profiles/ folder."""
    shape, storage = bench.WORKLOADS["singularities128"][0], bench.WORKLOADS["singularities128"][1]
    tile, variant = bench.tuned(shape, storage, 1, "singularities128")
    rec = dict(kernel_sha=bench.kernel_source_hash(), tile=list(tile or []), variant=variant,
               bytes_per_launch=123456.0)
    rec.update(over)
    (tmp_path / "profiles").mkdir(exist_ok=True)
    (tmp_path / "profiles" / "traffic_singularities128.json").write_text(json.dumps(rec))
    sha = bench.kernel_source_hash()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))               # records are read from here
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: sha)   # sources are still the repo's
    return storage


def test_traffic_record_used_only_while_current(tmp_path, monkeypatch):
    storage = _record(tmp_path, monkeypatch)
    assert bench.traffic_from_profile("singularities128", storage, 128 ** 3) == 123456.0
    # kernel sources changed since the counters were taken
    storage = _record(tmp_path, monkeypatch, kernel_sha="0" * 16)
    assert bench.traffic_from_profile("singularities128", storage, 128 ** 3) is None
    # taken on another tile or access variant than the benchmark now runs
    storage = _record(tmp_path, monkeypatch, variant=-1)
    assert bench.traffic_from_profile("singularities128", storage, 128 ** 3) is None
    # no record at all
    (tmp_path / "profiles" / "traffic_singularities128.json").unlink()
    assert bench.traffic_from_profile("singularities128", storage, 128 ** 3) is None


def test_two_pass_tuner_keeps_the_fastest_long_run(monkeypatch):
    from paper_0707_1299_amd import tune
    cands = [((64, 2, 2), 0), ((128, 2, 1), 2), ((256, 1, 1), 18), ((32, 4, 2), 16)]
    # short runs rank (128, 2, 1) first; the longer runs put (256, 1, 1) ahead
    short = {cands[0]: 1.00, cands[1]: 0.80, cands[2]: 0.85, cands[3]: 0.90}
    long = {cands[0]: 1.00, cands[1]: 0.86, cands[2]: 0.83, cands[3]: 0.88}
    calls = []

    def fake_run(name, steps, warmup, timing, choice=None):
        calls.append((choice, steps))
        t = (short if steps == 40 else long)[choice]
        return dict(kernel_ms=t * 0.9, ms_per_step=t, achieved_GBs=1.0), None

    saved = {}
    monkeypatch.setattr(tune, "candidates", lambda shape, storage: list(cands))
    monkeypatch.setattr(tune, "save", lambda shape, storage, nb, entry, tag=None: saved.update(entry, tag=tag))
    monkeypatch.setattr(bench, "run_workload", fake_run)
    bench.tune_workload("colloids256_fp32", steps=40, refine=2)
    assert [c for c, s in calls if s == 40] == cands                         # every candidate once
    assert sorted(c for c, s in calls if s == 200) == sorted([cands[1], cands[2]])   # the two fastest again
    assert saved["tile"] == [256, 1, 1] and saved["variant"] == 18 and saved["tag"] == "colloids256_fp32"
