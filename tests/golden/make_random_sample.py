"""Write random_sample.json: oracle picks of 17 wavelengths of each of the 30
random stress configurations (workloads.random_stress_config, seeds
1000-1029: random models outside the workloads' recipes, N 1-40, with
low-velocity layers and half-spaces slower than some layers), spread evenly
over each configuration's flattened wavelength list (those whose thickest
layer has k h <= 300: beyond about 350 the oracle's plain cosh and sinh
products overflow FP64).  The picks come from
oracle.dispersion_point (dense complex LU in FP64, linear scan, bisection)
alone.

Usage: python tests/golden/make_random_sample.py [processes]
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

SEEDS = range(1000, 1030)
PER_SEED = 17


KH_MAX = 300.0  # the oracle's unscaled cosh/sinh products overflow FP64 near k h = 350


def picks_of(seed: int):
    """(model, wavelength index) of the sampled wavelengths of one
    configuration, among those whose thickest layer has k h <= KH_MAX."""
    wl = WL.random_stress_config(seed)
    pairs = [(mi, wi) for mi, l in enumerate(wl.lambdas) for wi in range(len(l))
             if 2.0 * np.pi / l[wi] * (wl.models[mi].h.max() if wl.models[mi].n_layers else 0.0) <= KH_MAX]
    sel = np.linspace(0, len(pairs) - 1, PER_SEED).round().astype(int)
    return [pairs[i] for i in sel]


def _point(args):
    seed, mi, wi = args
    wl = WL.random_stress_config(seed)
    p = O.dispersion_point(float(wl.lambdas[mi][wi]), wl.c_test, wl.models[mi])
    return seed, mi, wi, p.idx, p.status, p.c_ref


def main():
    os.environ["OMP_NUM_THREADS"] = "1"
    tasks = [(s, mi, wi) for s in SEEDS for mi, wi in picks_of(s)]
    with mp.get_context("fork").Pool(int(sys.argv[1]) if len(sys.argv) > 1 else os.cpu_count()) as pool:
        pts = pool.map(_point, tasks, chunksize=1)
    out = {"source": "oracle.dispersion_point (dense LU, FP64) on workloads.random_stress_config",
           "cases": [{"seed": s, "model": mi, "lambda_index": wi, "idx": i, "status": st, "c_ref": cr}
                     for s, mi, wi, i, st, cr in pts]}
    with open(os.path.join(HERE, "random_sample.json"), "w") as f:
        json.dump(out, f)
        f.write("\n")
    print(f"{len(pts)} wavelengths, {sum(1 for p in pts if p[3] < 0)} without a pick", flush=True)


if __name__ == "__main__":
    main()
