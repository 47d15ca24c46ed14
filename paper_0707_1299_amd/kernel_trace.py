"""Per-kernel statistics of a rocprofv3 kernel trace, as a markdown table.

    python -m paper_0707_1299_amd.kernel_trace DIR [--match TEXT ...]

DIR is the output directory of one ``rocprofv3 --kernel-trace --stats -d DIR
-o run -- ...`` run; the dispatches are read from its results database
(``run_results.db``, view ``kernels``).  Durations are in microseconds; the
kernels are listed by total time.  With --match, only the kernels whose name
contains one of the texts are listed (the percentages stay those of the whole
trace).
"""
from __future__ import annotations

import argparse
import os
import sqlite3
import statistics

from .hbm_traffic import short_name


def stats(outdir):
    """[(kernel, calls, total us, avg us, min us, max us, median us, share of all kernel time)]."""
    cur = sqlite3.connect(os.path.join(outdir, "run_results.db")).cursor()
    durs = {}
    for name, d in cur.execute("select name, duration from kernels"):
        durs.setdefault(short_name(name), []).append(d / 1000.0)
    total = sum(sum(v) for v in durs.values())
    rows = [(k, len(v), sum(v), sum(v) / len(v), min(v), max(v), statistics.median(v), sum(v) / total)
            for k, v in durs.items()]
    return sorted(rows, key=lambda r: -r[2])


def table(rows, match=None):
    out = ["| kernel | calls | total us | avg us | min us | max us | median us | % |",
           "|---|---|---|---|---|---|---|---|"]
    for k, n, tot, avg, lo, hi, med, share in rows:
        if match and not any(m in k for m in match):
            continue
        out.append("| `%s` | %d | %.1f | %.3f | %.3f | %.3f | %.3f | %.2f |" % (k, n, tot, avg, lo, hi, med, 100 * share))
    return "\n".join(out)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("outdir")
    ap.add_argument("--match", nargs="*")
    a = ap.parse_args(argv)
    print(table(stats(a.outdir), a.match))


if __name__ == "__main__":
    main()
