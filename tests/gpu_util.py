"""Helpers shared by the GPU parity tests (comparison metrics and the
conversion of the library's deviation-form states to full populations)."""
import json
import os

import numpy as np
import torch

import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def thresholds(workload):
    """Frozen thresholds [4, 2] of a workload (+inf rows for absent sensors)."""
    data = json.load(open(os.path.join(GOLDEN, "thresholds.json")))
    t = np.full((4, 2), np.inf)
    rows = np.asarray(data[workload], np.float64)
    t[: rows.shape[0]] = rows
    return t


def to_f64(t):
    return t.detach().to("cpu", torch.float64).numpy() if torch.is_tensor(t) else np.asarray(t, np.float64)


def full_state(lat, q):
    """Full populations f = w rho0 + d of the current GPU state, FP64 numpy."""
    _, _, w = oracle.lattice(q)
    d = to_f64(lat.state)
    return w[:, None, None] * lat.cfg.rho0 + d


def deviation(f, q, rho0=1.0):
    _, _, w = oracle.lattice(q)
    return f - w[:, None, None] * rho0


def maxnorm(got, ref):
    """max |got - ref| / max |ref|."""
    got, ref = to_f64(got), to_f64(ref)
    den = np.abs(ref).max()
    return np.abs(got - ref).max() / (den if den > 0 else 1.0)


def flags_outside_band(gpu_flags, ref_flags, ref_sens, thr, mask, tol):
    """Compare flags on cells whose reference sensors are farther than
    tol * max|s| from every enabled threshold.  Returns (n_mismatch, n_excluded)."""
    gpu_flags, ref_flags = to_f64(gpu_flags), to_f64(ref_flags)
    near = np.zeros(ref_flags.shape, bool)
    for k in range(len(thr)):
        if mask & (1 << k):
            s = ref_sens[k]
            band = tol[k] * np.abs(s[np.isfinite(s)]).max() if np.isfinite(s).any() else 0
            for t in thr[k]:
                if np.isfinite(t):
                    near |= np.abs(s - t) <= band
    bad = (gpu_flags != ref_flags) & ~near
    return int(bad.sum()), int(near.sum())


def moment_errors(rho, ux, uy, ref, rho0=1.0):
    """Relative moment errors of a run: density max |d rho| / rho0 and velocity
    max |d u| / max |u| (the velocity vector field as a whole)."""
    rho, ux, uy = to_f64(rho), to_f64(ux), to_f64(uy)
    e_rho = np.abs(rho - ref[0]).max() / rho0
    du = np.hypot(ux - ref[1], uy - ref[2]).max()
    umax = np.hypot(ref[1], ref[2]).max()
    return e_rho, du / (umax if umax > 0 else 1.0)
