"""The committed oracle samples of the long runs (tests/golden/*_oracle_*.npz) are
consistent: written by the current oracle source (its sha256 is stored with
them), with node indices inside the lattice and arrays of matching sizes.  They
are produced by tests/golden/make_long_goldens.py, which calls only the oracle."""
import glob
import hashlib
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FILES = sorted(glob.glob(os.path.join(ROOT, "tests", "golden", "*_oracle_*.npz")))
SIZES = {"singularities128": 128, "colloids256": 256}


@pytest.mark.parametrize("path", FILES, ids=[os.path.basename(f) for f in FILES])
def test_oracle_sample_file(path):
    d = np.load(path, allow_pickle=False)
    sha = hashlib.sha256(open(os.path.join(ROOT, "oracle", "lbm_oracle.c"), "rb").read()).hexdigest()
    assert str(d["oracle_sha"]) == sha
    name = os.path.basename(path).split("_oracle_")[0]
    L = SIZES[name]
    steps = int(os.path.basename(path).split("_oracle_")[1].split(".")[0])
    assert int(d["steps"]) == steps
    nodes = d["nodes"]
    assert nodes.ndim == 1 and len(np.unique(nodes)) == len(nodes)
    assert nodes.min() >= 0 and nodes.max() < L ** 3
    assert d["u"].shape == (3, len(nodes)) and d["rho"].shape == (len(nodes),)
    assert np.all(np.isfinite(d["u"])) and float(d["umax"]) >= np.abs(d["u"]).max()
    assert d["df_sum"].shape == (19,) and d["c"].shape == (19, 3)
    assert d["U"].shape == d["pos"].shape and d["U"].shape[1] == 3
    # mass is conserved exactly by the method: the deviation sum stays at rounding level
    assert abs(float(d["df_sum"].sum())) < 1e-9
