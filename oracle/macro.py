"""Macroscopic (class-1) sensors from moment fields with central finite
differences: the counterparts the paper compares its kinetic class-1 sensors
with (Sec. III.A, eqs. sensor-TauNS-mac, sensor-C-mac, sensor-S-mac, the
rate-of-strain and heat-flux forms; Sec. IV: central differences).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Fields are [ny][nx] (x fastest).  d/dx a at cell j = (a[j+1] - a[j-1]) / (2 dx),
ghost cells by the boundary condition of the axis: 0 periodic (wrap), 1
zero-gradient (repeat the edge cell).  With A_ab = d_a u_b (a, b in {x, y}):
    tau  = -mu (A + A^T) - lambda (div u) I          |tau|_F
    C    = sqrt(D) |div u|
    S    = |A + A^T - (2/D)(div u) I|_F
    E    = |(A + A^T)/2|_F
    qH   = |u . tau|          ((u . tau)_b = sum_a u_a tau_ab)
    qF   = |kappa grad T|
    qNSF = |-kappa grad T + u . tau|
mu, lambda, kappa are multiplied by the cell's density when per_rho.
"""
import numpy as np

NAMES = ("tau", "c", "s", "e", "qh", "qf", "qnsf")


def _ddx(a, dx, bc, axis):
    n = a.shape[axis]
    if bc == 0:
        ap, am = np.roll(a, -1, axis), np.roll(a, 1, axis)
    else:
        idx = np.arange(n)
        ap = np.take(a, np.minimum(idx + 1, n - 1), axis)
        am = np.take(a, np.maximum(idx - 1, 0), axis)
    return (ap - am) / (2.0 * dx)


def macro_sensors(rho, ux, uy, T, mu, lam, kappa, dx=1.0, bc=(0, 0), per_rho=False, which=NAMES):
    """dict name -> [ny][nx] of the requested sensors (FP64)."""
    D = 2
    dxx = _ddx(ux, dx, bc[0], 1)       # d_x u_x
    dxy = _ddx(uy, dx, bc[0], 1)       # d_x u_y
    dyx = _ddx(ux, dx, bc[1], 0)       # d_y u_x
    dyy = _ddx(uy, dx, bc[1], 0)       # d_y u_y
    div = dxx + dyy
    scale = rho if per_rho else 1.0
    m, l, k = mu * scale, lam * scale, kappa * scale
    # symmetric part A + A^T
    sxx, syy, sxy = 2.0 * dxx, 2.0 * dyy, dxy + dyx
    txx = -m * sxx - l * div
    tyy = -m * syy - l * div
    txy = -m * sxy
    out = {}
    out["tau"] = np.sqrt(txx ** 2 + tyy ** 2 + 2.0 * txy ** 2)
    out["c"] = np.sqrt(D) * np.abs(div)
    out["s"] = np.sqrt((sxx - 2.0 / D * div) ** 2 + (syy - 2.0 / D * div) ** 2 + 2.0 * sxy ** 2)
    out["e"] = 0.5 * np.sqrt(sxx ** 2 + syy ** 2 + 2.0 * sxy ** 2)
    qhx, qhy = ux * txx + uy * txy, ux * txy + uy * tyy
    out["qh"] = np.hypot(qhx, qhy)
    if T is not None:
        gx, gy = _ddx(T, dx, bc[0], 1), _ddx(T, dx, bc[1], 0)
        out["qf"] = np.hypot(k * gx, k * gy)
        out["qnsf"] = np.hypot(-k * gx + qhx, -k * gy + qhy)
    return {n: out[n] for n in which}
