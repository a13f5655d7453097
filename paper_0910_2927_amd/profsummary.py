"""Summaries of rocprofv3 result databases for this library's kernels.

rocprofv3 (ROCm 7) writes its results as a SQLite database
(``<dir>/**/<name>_results.db``).  This reads the ``kernels`` view (kernel
trace) or the ``counters_collection`` view (``--pmc`` runs) with the
standard library only and prints one Markdown table row per kernel
instance:

    python -m paper_0910_2927_amd.profsummary trace DIR [--after NAME]
        | kernel | dispatches | total ms | average us | share % |
    python -m paper_0910_2927_amd.profsummary counters DIR [--after NAME]
        | kernel grid=G | counter | dispatches | average value per dispatch |
    python -m paper_0910_2927_amd.profsummary batched DIR
        | kernel | dispatches | total ms | average us |   (the batched solver's
                                                      kernels, k_b*, only)

--after NAME keeps the dispatches from the first one whose kernel name
contains NAME on (e.g. k_fom_poles: a solve's first restart cycle ends with
it, and the deflation eigensolve before it never launches it).  Kernel
names are shortened: complex vector types become double2 / float2 and the
argument lists are dropped.
"""
from __future__ import annotations

import argparse
import glob
import os
import re
import sqlite3
from collections import OrderedDict


def short(name: str) -> str:
    n = name.replace("HIP_vector_type<double, 2u>", "double2").replace("HIP_vector_type<float, 2u>", "float2")
    n = n.replace("(anonymous namespace)::", "")
    n = re.sub(r"\(.*", "", n)
    return n.replace("void ", "").replace("sk::", "").strip()


def find_db(path: str) -> str:
    if path.endswith(".db"):
        return path
    dbs = glob.glob(os.path.join(path, "**", "*_results.db"), recursive=True)
    if not dbs:
        raise SystemExit(f"no *_results.db under {path}")
    return dbs[0]


def _after(rows, name_idx, after):
    if not after:
        return rows
    for i, r in enumerate(rows):
        if after in r[name_idx]:
            return rows[i:]
    return []


def trace(db: str, after: str | None = None):
    cur = sqlite3.connect(db).cursor()
    rows = cur.execute("select name, duration from kernels order by start").fetchall()
    rows = _after(rows, 0, after)
    agg = OrderedDict()
    for name, dur in rows:
        a = agg.setdefault(short(name), [0, 0.0])
        a[0] += 1
        a[1] += dur
    return agg


def counters(db: str, after: str | None = None):
    cur = sqlite3.connect(db).cursor()
    rows = cur.execute("select kernel_name, counter_name, value, grid_size from counters_collection "
                       "order by start").fetchall()
    rows = _after(rows, 0, after)
    agg = OrderedDict()
    for name, cname, value, grid in rows:
        a = agg.setdefault((f"{short(name)} grid={grid}", cname), [0, 0.0])
        a[0] += 1
        a[1] += value
    return agg


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("mode", choices=["trace", "counters", "batched"])
    ap.add_argument("path", help="rocprofv3 output directory or database")
    ap.add_argument("--after", default=None)
    a = ap.parse_args(argv)
    db = find_db(a.path)
    if a.mode in ("trace", "batched"):
        agg = trace(db, a.after)
        tot = sum(v[1] for v in agg.values()) or 1.0
        for k, (c, d) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
            if a.mode == "batched" and not k.startswith("k_b"):
                continue
            share = f" {100 * d / tot:.1f} |" if a.mode == "trace" else ""
            print(f"| {k} | {c} | {d / 1e6:.3f} | {d / c / 1e3:.2f} |{share}")
    else:
        for (k, cn), (c, v) in counters(db, a.after).items():
            print(f"| {k} | {cn} | {c} | {v / c:.1f} |")


if __name__ == "__main__":
    main()
