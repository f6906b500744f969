"""Write the oracle's expected values for a wavelength where a mode and a pole
of det K lie within two grid steps of each other.

The wavelength comes from the seeded serving workload: request 21269 of the
Poisson trace at 2000 req/s (arrival seed 55; chain choices and random-walk
steps from PCG64(56); 64 chains from chain_bases(64, 5)), its wavelength 124,
on the serving grid (50-1000 m/s at 0.1 m/s).  Its first sign change is a
mode at about 67.98 m/s, and the next, one grid step later, is a pole of a
low-velocity layer (beta 45.5 m/s): between them an FP32 determinant takes the
wrong sign.  The file stores the model, the wavelength, and the oracle's
pick, status, bisection root and zero/pole class (calls only oracle/ and
workloads/).

Usage: python tests/golden/make_split_pole_case.py
"""
from __future__ import annotations

import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
from oracle import propagator as PR  # noqa: E402
import workloads as WL  # noqa: E402

REQUEST, WAVELENGTH = 21269, 124


def serving_request(index: int):
    bases = WL.chain_bases(64, 5)
    times = WL.poisson_arrivals(2000.0, 11.0, 55)
    rng = np.random.Generator(np.random.PCG64(56))
    pick = rng.integers(0, len(bases), size=len(times))
    state = [b.model for b in bases]
    for i in range(index + 1):
        ch = int(pick[i])
        state[ch] = WL.chain_step(rng, state[ch])
    return state[int(pick[index])], bases[int(pick[index])].lambdas


def main():
    model, lambdas = serving_request(REQUEST)
    lam = float(lambdas[WAVELENGTH])
    c = WL.serving_grid()
    p = O.dispersion_point(lam, c, model)
    cls, c_sec = PR.classify(lam, c, p.idx, model)
    nxt = O.first_sign_change(2 * np.pi / lam, c[p.idx:], model)[0] + p.idx
    out = {
        "source": f"serving trace request {REQUEST}, wavelength {WAVELENGTH}; oracle/ only",
        "h": model.h.tolist(), "alpha": model.alpha.tolist(), "beta": model.beta.tolist(),
        "rho": model.rho.tolist(), "lambda": lam,
        "idx": p.idx, "status": p.status, "c_ref": repr(p.c_ref), "class": cls,
        "next_idx": int(nxt), "next_class": PR.classify(lam, c, int(nxt), model)[0],
    }
    path = os.path.join(HERE, "split_pole_case.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {path}: idx {p.idx} ({['MODE', 'POLE'][cls]}), next change {nxt} "
          f"({['MODE', 'POLE'][out['next_class']]})")


if __name__ == "__main__":
    main()
