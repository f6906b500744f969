"""Write the oracle's expected values for the large parity cases.

Calls only oracle/ and workloads/ (never the HIP library).  Output files:

  fine_scale.json   all 1000 wavelengths of the 20-layer fine-scale case
                    (c 50-1200 m/s at 0.01 m/s, 115,001 values)
  batch_sample.json 64 models of the 4096-model batch case, stratified by
                    layer count and inversion, all their wavelengths

Each entry stores the grid index of the first sign change (Algorithm 1), the
status, and the bisection root (17 significant digits).

Usage: python tests/golden/make_golden.py [fine|batch|all] [--workers P]
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
os.environ.setdefault("OMP_NUM_THREADS", "1")

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
import workloads as WL  # noqa: E402


def _point(args):
    lam, c_test, model = args
    p = O.dispersion_point(lam, c_test, model)
    return p.idx, p.status, p.c_ref, p.evals


def batch_sample_indices(wl, n: int = 64):
    """Stratified sample: models sorted by (inverted, N, index), n evenly spaced."""
    keys = sorted(range(len(wl.models)),
                  key=lambda i: (wl.meta["inverted"][i], wl.models[i].n_layers, i))
    pos = np.linspace(0, len(keys) - 1, n).round().astype(int)
    return sorted(keys[p] for p in pos)


def run(tasks, workers):
    with mp.Pool(workers) as pool:
        return pool.map(_point, tasks, chunksize=1)


def make_fine(workers):
    wl = WL.fine_scale_case()
    m = wl.models[0]
    lams = wl.lambdas[0]
    # deepest first so that the pool stays busy at the end
    order = np.argsort(-lams)
    res = run([(float(lams[i]), wl.c_test, m) for i in order], workers)
    out = [None] * len(lams)
    for i, r in zip(order, res):
        out[i] = r
    return {"workload": wl.name, "source": "oracle.dispersion_point (dense LU, FP64)",
            "idx": [int(r[0]) for r in out], "status": [int(r[1]) for r in out],
            "c_ref": [repr(float(r[2])) for r in out], "evals": int(sum(r[3] for r in out))}


def make_batch(workers):
    wl = WL.batch_case()
    sel = batch_sample_indices(wl)
    tasks, owner = [], []
    for mi in sel:
        for j, lam in enumerate(wl.lambdas[mi]):
            tasks.append((float(lam), wl.c_test, wl.models[mi]))
            owner.append((mi, j))
    order = sorted(range(len(tasks)), key=lambda t: -tasks[t][0] * tasks[t][2].n_layers)
    res = run([tasks[t] for t in order], workers)
    by = {}
    for t, r in zip(order, res):
        by[owner[t]] = r
    models = []
    for mi in sel:
        W = len(wl.lambdas[mi])
        rs = [by[(mi, j)] for j in range(W)]
        models.append({"model": int(mi), "idx": [int(r[0]) for r in rs], "status": [int(r[1]) for r in rs],
                       "c_ref": [repr(float(r[2])) for r in rs]})
    return {"workload": wl.name, "source": "oracle.dispersion_point (dense LU, FP64)",
            "models": models, "evals": int(sum(r[3] for r in res))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", nargs="?", default="all", choices=["fine", "batch", "all"])
    ap.add_argument("--workers", type=int, default=os.cpu_count())
    a = ap.parse_args()
    if a.which in ("fine", "all"):
        t = time.time()
        d = make_fine(a.workers)
        with open(os.path.join(HERE, "fine_scale.json"), "w") as f:
            json.dump(d, f, separators=(",", ":"))
        print(f"fine_scale.json: {len(d['idx'])} wavelengths, {d['evals']} evals, {time.time() - t:.0f} s", flush=True)
    if a.which in ("batch", "all"):
        t = time.time()
        d = make_batch(a.workers)
        with open(os.path.join(HERE, "batch_sample.json"), "w") as f:
            json.dump(d, f, separators=(",", ":"))
        print(f"batch_sample.json: {len(d['models'])} models, {d['evals']} evals, {time.time() - t:.0f} s", flush=True)


if __name__ == "__main__":
    main()
