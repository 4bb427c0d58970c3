"""Writes tests/golden/oracle_values.json: CPU-oracle TWED values for the
seeded workloads whose oracle run is too long for a test (up to minutes).

Calls only oracle/ (and the seeded generators).  Regenerate with

    python tests/golden/make_golden.py [--jobs N]

Inputs marked "f32" are generated in FP64, rounded once to FP32 and widened
back, so the value is the exact-arithmetic reference for the FP32 GPU paths.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2007_16135_amd import synth  # noqa: E402

CASES = [
    # name, generator, n, prefix, input rounding
    ("walk1d_n1000", "single_pair_1d", 1000, None, "f64"),
    ("walk1d_n1000_f32", "single_pair_1d", 1000, None, "f32"),
    ("walk3d_n100000", "single_pair_3d", 100000, None, "f64"),
    ("walk3d_n100000_f32", "single_pair_3d", 100000, None, "f32"),
    ("walk3d_n100000_prefix10000", "single_pair_3d", 100000, 10000, "f64"),
    ("walk3d_n100000_prefix10000_f32", "single_pair_3d", 100000, 10000, "f32"),
    ("walk8d_n1000000_prefix10000_f32", "single_pair_8d", 1000000, 10000, "f32"),
    ("walk8d_n1000000_prefix10000", "single_pair_8d", 1000000, 10000, "f64"),
    ("walk8d_n1000000_prefix20000_f32", "single_pair_8d", 1000000, 20000, "f32"),
]


def run_case(case):
    name, gen, n, prefix, rnd = case
    c = getattr(synth, gen)(n)
    if prefix:
        c = c.prefix(prefix)
    if rnd == "f32":
        c = c.astype(np.float32).astype(np.float64)
    t0 = time.time()
    v = oracle.get().twed(c.A, c.TA, c.B, c.TB, c.nu, c.lam, c.p, rows=True)
    return {"name": name, "generator": f"synth.{gen}({n})", "prefix": prefix, "inputs": rnd,
            "nu": c.nu, "lambda": c.lam, "p": c.p, "dim": c.dim, "nA": len(c.TA), "nB": len(c.TB),
            "value": v, "oracle": "twed_oracle_rows (FP64)", "seconds": round(time.time() - t0, 2)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=4)
    a = ap.parse_args()
    oracle.get()  # build once before forking workers
    with cf.ProcessPoolExecutor(max_workers=a.jobs) as ex:
        res = list(ex.map(run_case, CASES))
    out = {"about": "FP64 CPU-oracle values of seeded synthetic workloads; written by "
                    "tests/golden/make_golden.py, which calls only oracle/.",
           "cases": res}
    with open(os.path.join(HERE, "oracle_values.json"), "w") as f:
        json.dump(out, f, indent=1)
    for r in res:
        print(r["name"], repr(r["value"]), r["seconds"], "s")


if __name__ == "__main__":
    main()
