"""Writes thresholds.json: the refinement thresholds of each workload, frozen
from the FP64 oracle at the workload's final step, rounded to two significant
digits.  Smooth fields (C1, C2): theta1, theta2 = the 90th and 99th
percentiles of each sensor over all cells.  Riemann problem (C3): most cells
sit exactly at a uniform equilibrium there (sensors at round-off), so
theta1, theta2 = 1 % and 10 % of each sensor's maximum; likewise for its
double-distribution form (C4, five sensors with S_QE).  Calls only the oracle
and the seeded input generators.

    python tests/golden/make_thresholds.py [C1] [C2] [C3] [C4]
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2603_13618_amd import inputs  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "thresholds.json")


def sig2(x):
    return float(f"{x:.2g}")


def pct(sens, nsens):
    return [[sig2(np.percentile(sens[k], 90)), sig2(np.percentile(sens[k], 99))]
            for k in range(nsens)]


def c1():
    rho, ux, uy = inputs.double_shear_layer(128)
    out = oracle.run(9, oracle.equilibrium(9, rho, ux, uy), 500, tau=0.55)
    return pct(out["sens"], 3)


def c2():
    rho, ux, uy = inputs.smooth_random(4096, seed=0, cutoff=16)
    out = oracle.run(9, oracle.equilibrium(9, rho, ux, uy), 100, tau=0.52)
    return pct(out["sens"], 3)


def c3():
    n = 2048
    rho, ux, uy, T, states = inputs.riemann_quadrants(n, seed=0)
    dx = 1.0 / n
    dt = inputs.riemann_dt(states, dx)
    out = oracle.run(25, oracle.equilibrium(25, rho, ux, uy, T), 200, mu=1e-3, dt=dt, dx=dx,
                     bc=(1, 1))
    return [[sig2(0.01 * out["sens"][k].max()), sig2(0.1 * out["sens"][k].max())]
            for k in range(4)]


def c4():
    # the Riemann problem with the double distribution (air: gamma = 1.4,
    # Pr = 0.71); five sensors, the fifth the quasi-equilibrium sensor
    n = 2048
    rho, ux, uy, T, states = inputs.riemann_quadrants(n, seed=0)
    dx = 1.0 / n
    dt = inputs.riemann_dt(states, dx, gamma=1.4)
    out = oracle.ddf_run(oracle.ddf_equilibrium(rho, ux, uy, T, 1.4), 200, 1e-3, dt, dx,
                         bc=(1, 1), gamma=1.4, prandtl=0.71)
    return [[sig2(0.01 * out["sens"][k].max()), sig2(0.1 * out["sens"][k].max())]
            for k in range(5)]


if __name__ == "__main__":
    which = sys.argv[1:] or ["C1"]
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for w in which:
        data[w] = {"C1": c1, "C2": c2, "C3": c3, "C4": c4}[w]()
        print(w, data[w], flush=True)
    data["_recipe"] = ("per sensor (S_KL, S_NEQ, S_PI[, S_Q]): [90th, 99th] percentile over all "
                       "cells at the final step of the FP64 oracle run, 2 significant digits")
    json.dump(data, open(OUT, "w"), indent=1, sort_keys=True)
