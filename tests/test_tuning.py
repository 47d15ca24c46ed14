"""Host logic of the tile / variant cache (no GPU): shape entries, per-workload tagged entries
with fallback, and the candidate list's rules (tiles no wider than twice the box, whole-wave
tile rows for boxes of 4 GiB or more, lane mode as an FP16 variant)."""
import json

from paper_0707_1299_amd import tune


def test_lookup_tag_falls_back_to_shape_entry(tmp_path, monkeypatch):
    cache = tmp_path / "cache.json"
    monkeypatch.setattr(tune, "CACHE", str(cache))
    assert tune.lookup((16, 16, 16), "fp32") is None
    tune.save((16, 16, 16), "fp32", 1, dict(tile=[64, 2, 2], variant=16))
    tune.save((16, 16, 16), "fp32", 1, dict(tile=[32, 4, 2], variant=2), tag="crowded")
    assert tune.lookup((16, 16, 16), "fp32") == ((64, 2, 2), 16)
    assert tune.lookup((16, 16, 16), "fp32", tag="crowded") == ((32, 4, 2), 2)
    assert tune.lookup((16, 16, 16), "fp32", tag="other") == ((64, 2, 2), 16)
    assert tune.lookup((16, 16, 16), "fp64") is None
    assert tune.lookup((16, 16, 16), "fp32", nboxes=2) is None
    keys = json.load(open(cache))
    assert tune.key((16, 16, 16), "fp32", 1, "crowded") in keys


def test_candidates_rules():
    small = tune.candidates((32, 32, 32), "fp32")
    assert all(t[0] <= 64 for t, _ in small)
    assert all(v & 32 == 0 for _, v in small)                  # lane mode is FP16 only
    big32 = tune.candidates((512, 512, 512), "fp32")             # 10 GB box: >= 64 lanes along x
    assert big32 and all(t[0] >= 64 for t, _ in big32)
    big16 = tune.candidates((512, 512, 512), "fp16")             # 5 GB box
    for t, v in big16:
        lanes = t[0] if v & 32 else t[0] // 2
        assert lanes >= 64
    assert any(v & 32 for _, v in big16) and any(not v & 32 for _, v in big16)
    odd16 = tune.candidates((16, 16, 33), "fp16")                # odd nx: one node per lane only
    assert all(v & 32 == 0 for _, v in odd16)
    # the kernel without the tile loop (bit 128) only with one tile per block, and offered for it
    assert all(not (v >> 2) & 3 for _, v in small if v & 128)
    assert {v & ~128 for _, v in small if v & 128} == {v for _, v in small if not (v >> 2) & 3 and not v & 128}
