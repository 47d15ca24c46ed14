"""HBM bytes per launch of the fused step kernel from rocprofv3 counter runs.

    python -m paper_0707_1299_amd.hbm_traffic --workload singularities128 \
        --fetch DIR --write DIR --copy-fetch DIR --copy-write DIR

Each DIR is the output directory of one ``rocprofv3 --pmc FETCH_SIZE`` (or
``WRITE_SIZE``) run with ``-o run``: the step kernel's runs come from
``bench.py --workload W``, the calibration runs from ``bench.py
--copy-calibration`` (10 torch copies and 10 copies by the library's
streaming probe, 512 MiB each).  FETCH_SIZE and WRITE_SIZE are given in KiB
per dispatch; each is scaled by (bytes a copy must move) / (what the counter
reads for the probe's copy), and the kernel's traffic is the sum of the two
scaled medians.  The result goes to profiles/traffic_<workload>.json with the
hash of the kernel sources and the tile / variant it was taken with;
bench.py reports it as roofline.traffic only while all three still match.
"""
from __future__ import annotations

import argparse
import json
import os
import sqlite3
import statistics
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_BYTES = 1 << 29


def short_name(name):
    """Kernel name without its trailing parameter list."""
    if not name.endswith(")"):
        return name
    depth = 0
    for i in range(len(name) - 1, -1, -1):
        depth += {")": 1, "(": -1}.get(name[i], 0)
        if depth == 0:
            return name[:i]
    return name


def per_kernel(outdir, counter):
    """{kernel name without arguments: [counter value per dispatch]} from a rocprofv3 results database."""
    db = os.path.join(outdir, "run_results.db")
    cur = sqlite3.connect(db).cursor()
    out = {}
    for name, v in cur.execute("select name, counter_value from pmc_events where counter_name=?", (counter,)):
        out.setdefault(short_name(name), []).append(v)
    return out


def pick(d, needle):
    names = [k for k in d if needle in k]
    if not names:
        raise SystemExit("no dispatch of a kernel named *%s* in the counter data" % needle)
    return names[0], d[names[0]]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="singularities128")
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--copy-fetch", required=True)
    ap.add_argument("--copy-write", required=True)
    ap.add_argument("--record", default=None,
                    help="name of the record (profiles/traffic_<record>.json); default the workload's name")
    a = ap.parse_args()
    sys.path.insert(0, ROOT)
    import bench

    shape, storage = bench.WORKLOADS[a.workload][0], bench.WORKLOADS[a.workload][1]
    kib = COPY_BYTES / 1024
    cf, cw = per_kernel(a.copy_fetch, "FETCH_SIZE"), per_kernel(a.copy_write, "WRITE_SIZE")
    _, pf = pick(cf, "k_copy16")
    _, pw = pick(cw, "k_copy16")
    scale_f, scale_w = kib / statistics.median(pf), kib / statistics.median(pw)
    torch_copy = {}
    if any("copyBuffer" in k for k in cf):
        tf, tw = pick(cf, "copyBuffer")[1], pick(cw, "copyBuffer")[1]
        torch_copy = dict(fetch_kib=statistics.median(tf), write_kib=statistics.median(tw),
                          scale_fetch=kib / statistics.median(tf), scale_write=kib / statistics.median(tw))
    kf, kw = per_kernel(a.fetch, "FETCH_SIZE"), per_kernel(a.write, "WRITE_SIZE")
    name, f = pick(kf, "k_lattice")
    _, w = pick(kw, "k_lattice")
    f, w = statistics.median(f), statistics.median(w)
    nboxes = bench.WORKLOADS[a.workload][4] if bench.WORKLOADS[a.workload][3] == "boxes" else 1
    alg = bench.BYTES_PER_NODE[storage] * shape[0] * shape[1] * shape[2] * nboxes
    traffic = (f * scale_f + w * scale_w) * 1024
    tile, variant = bench.tuned(shape, storage, nboxes, a.workload)
    out = dict(workload=a.workload, record=a.record or a.workload, kernel=name, kernel_sha=bench.kernel_source_hash(),
               tile=list(tile) if tile else None, variant=variant,
               fetch_kib_per_dispatch=f, write_kib_per_dispatch=w, dispatches=len(kf[name]),
               calibration="lb_copy_probe (16-byte non-temporal copy), %d bytes read and written" % COPY_BYTES,
               copy_fetch_kib=statistics.median(pf), copy_write_kib=statistics.median(pw),
               scale_fetch=scale_f, scale_write=scale_w, torch_copy=torch_copy,
               bytes_per_launch=traffic, algorithmic_bytes_per_launch=alg, traffic_over_algorithmic=traffic / alg)
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % (a.record or a.workload))
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
