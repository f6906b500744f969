"""Write split_misses.json: oracle picks of the wavelengths of the random
stress configurations on which an FP32 sweep with FP64 window checks alone
missed Algorithm 1's first sign change (FP32 saw none of an even number of
changes between two FP64-checked points).  Each case is named by its
configuration seed, model and wavelength index in
workloads.random_stress_config; the picks come from oracle.dispersion_point
(dense complex LU in FP64, linear scan, bisection) alone, with the FP64 noise
band tested at both bracket points.

Usage: python tests/golden/make_split_misses.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
import workloads as WL  # noqa: E402

# (seed, model, wavelength index)
CASES = [(1016, 3, 230), (1028, 55, 230)]


def main():
    out = {"source": "oracle.dispersion_point (dense LU, FP64) on workloads.random_stress_config",
           "cases": []}
    for seed, mi, wi in CASES:
        wl = WL.random_stress_config(seed)
        m, lam, c = wl.models[mi], float(wl.lambdas[mi][wi]), wl.c_test
        p = O.dispersion_point(lam, c, m)
        band = [bool(O.in_noise_band(lam, float(c[i]), m)) for i in (p.idx - 1, p.idx)] if p.idx > 0 else []
        out["cases"].append({"seed": seed, "model": mi, "lambda_index": wi, "lambda": lam, "n_layers": m.n_layers,
                             "beta_hs": float(m.beta[-1]), "idx": p.idx, "status": p.status,
                             "c_t": p.c_t, "c_ref": p.c_ref, "bracket_in_noise_band": band})
        print(out["cases"][-1], flush=True)
    with open(os.path.join(HERE, "split_misses.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
