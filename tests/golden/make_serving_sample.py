"""Write serving_sample.json: oracle picks of every wavelength of 64 requests
sampled evenly from the serving trace (workloads.serving_trace at 2000 req/s
over 11 s, 1 s of it warm-up; request grid workloads.serving_grid(), 9,501
velocities).  The picks come from oracle.dispersion_point (dense complex LU
in FP64, linear scan, bisection) alone.

Usage: python tests/golden/make_serving_sample.py [processes]
"""
import json
import multiprocessing as mp
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
import workloads as WL  # noqa: E402

RATE, DURATION, SEED, N_SAMPLE = 2000.0, 11.0, 55, 64


def sample_indices(n_requests: int) -> list:
    return [int(i) for i in np.linspace(0, n_requests - 1, N_SAMPLE).round()]


def _point(args):
    lam, model = args
    p = O.dispersion_point(lam, WL.serving_grid(), model)
    return p.idx, p.status, p.c_ref


def main():
    os.environ["OMP_NUM_THREADS"] = "1"
    times, reqs = WL.serving_trace(RATE, DURATION, SEED)
    pick = sample_indices(len(times))
    tasks = [(float(l), reqs[i][0]) for i in pick for l in reqs[i][1]]
    with mp.get_context("fork").Pool(int(sys.argv[1]) if len(sys.argv) > 1 else os.cpu_count()) as pool:
        pts = pool.map(_point, tasks, chunksize=4)
    out = {"source": "oracle.dispersion_point (dense LU, FP64) on workloads.serving_trace",
           "rate": RATE, "duration": DURATION, "seed": SEED, "n_requests": len(times), "requests": []}
    k = 0
    for i in pick:
        W = len(reqs[i][1])
        sl = pts[k:k + W]
        k += W
        out["requests"].append({"index": i, "n_layers": reqs[i][0].n_layers, "idx": [p[0] for p in sl],
                                "status": [p[1] for p in sl], "c_ref": [p[2] for p in sl]})
    with open(os.path.join(HERE, "serving_sample.json"), "w") as f:
        json.dump(out, f)
        f.write("\n")
    print(f"{len(pick)} requests, {len(tasks)} wavelengths", flush=True)


if __name__ == "__main__":
    main()
