"""Grids whose element offsets pass 2^31, checked against the FP64 oracle on
sampled patches (the domain-of-dependence windows of test_gpu_fullsize).

D2Q9 FP32 at 16384^2 in both population layouts: plane-major offsets reach
8 x 16384^2 = 2.1e9 elements, row-interleaved ones y * 9 * 16384 = 2.4e9.
The double distribution at 8192^2 stores 50 planes: 3.3e9 elements in either
layout.  Bars as in the full-size tests (moments 1e-5, sensors 1e-3 of the
patch maximum, flags outside the threshold band bit-exact).
"""
import numpy as np
import pytest
import torch

from paper_2603_13618_amd import inputs, lks, workloads

from gpu_util import flags_outside_band, to_f64

pytestmark = pytest.mark.gpu

P = 16
# integer wavenumbers, so the fields are periodic on the grid and can be
# evaluated at window coordinates outside [0, n)
KX = (397, 451, 503)
KY = (389, 523, 419)


def _fields(n, xs, ys):
    """rho, ux, uy on the points (xs, ys) of an n x n periodic grid (separable
    products of sines, wavelengths of 30 - 40 cells)."""
    tx, ty = 2.0 * np.pi * np.asarray(xs, np.float64) / n, 2.0 * np.pi * np.asarray(ys, np.float64) / n
    rho = 1.0 + 0.02 * np.outer(np.cos(KY[0] * ty), np.sin(KX[0] * tx + 0.3))
    ux = 0.03 * np.outer(np.sin(KY[1] * ty), np.cos(KX[1] * tx))
    uy = 0.03 * np.outer(np.sin(KY[2] * ty), np.cos(KX[2] * tx + 0.1))
    return rho, ux, uy


def _dpatch(t, y0, x0):
    return to_f64(t[..., y0:y0 + P, x0:x0 + P])


def _window(orc, n, x0, y0, steps, tau, thr, mask):
    R = steps + 1
    rho, ux, uy = _fields(n, np.arange(x0 - R, x0 + P + R), np.arange(y0 - R, y0 + P + R))
    out = orc.run(9, orc.equilibrium(9, rho, ux, uy), steps, tau=tau, thr=thr, mask=mask)
    sl = (slice(R, R + P), slice(R, R + P))
    return {"mom": out["mom"][(slice(None),) + sl], "sens": out["sens"][(slice(None),) + sl],
            "flags": out["flags"][sl]}


@pytest.mark.parametrize("layout", ["rows", "planes"])
def test_d2q9_16384_fp32_sampled(orc, layout):
    n, steps, tau = 16384, 8, 0.6
    mask = lks.S_KL | lks.S_NEQ | lks.S_PI
    patches = ((0, 0), (8000, 12001), (n - P, n - P))
    # thresholds inside the sensors' range, from the first patch's reference
    probe = _window(orc, n, *patches[0], steps, tau, None, 0)
    thr = np.full((4, 2), np.inf)
    for k in range(3):
        thr[k] = np.quantile(probe["sens"][k], [0.3, 0.7])
    refs = [_window(orc, n, x0, y0, steps, tau, thr, mask) for x0, y0 in patches]
    rho, ux, uy = _fields(n, np.arange(n), np.arange(n))
    lat = lks.Lattice(9, n, n, "f32", tau=tau, thr=thr, flag_mask=mask, max_steps=steps, layout=layout)
    lat.init(rho, ux, uy)
    del rho, ux, uy
    lat.step(steps)
    torch.cuda.synchronize()
    assert lat.check() == 0
    r, u, v, _ = lat.moments()
    for (x0, y0), ref in zip(patches, refs):
        m = ref["mom"]
        e_rho = np.abs(_dpatch(r, y0, x0) - m[0]).max()
        e_u = np.hypot(_dpatch(u, y0, x0) - m[1], _dpatch(v, y0, x0) - m[2]).max() / np.hypot(m[1], m[2]).max()
        es = [np.abs(_dpatch(lat.sensors[k], y0, x0) - ref["sens"][k]).max() / np.abs(ref["sens"][k]).max()
              for k in range(3)]
        print(f"{layout} patch ({x0},{y0}): rho {e_rho:.2e} u {e_u:.2e} sensors "
              + " ".join(f"{e:.2e}" for e in es), flush=True)
        assert e_rho <= 1e-5 and e_u <= 1e-5
        assert max(es) <= 1e-3
        bad, excl = flags_outside_band(_dpatch(lat.flags, y0, x0), ref["flags"], ref["sens"], thr, mask,
                                       [max(e, 1e-6) for e in es] + [0])
        assert bad == 0, (bad, excl)
    # the FP64 sums see every cell: mass conserved to FP32 rounding
    s = to_f64(lat.sums)
    assert np.abs(s[:, 0] / (n * n) - s[0, 0] / (n * n)).max() < 1e-6


def test_ddf_8192_fp32_sampled(orc):
    wl = workloads.RIEMANN_2048_DDF
    n, steps, mu, gamma, pr = 8192, 4, wl["mu"], wl["gamma"], wl["prandtl"]
    thr, mask = np.asarray(wl["thr"]), wl["flag_mask"]
    thr5 = np.vstack([thr, [wl["thr_qe"]]])
    rho, ux, uy, T, states = inputs.riemann_quadrants(n, seed=0)
    dx = 1.0 / n
    dt = inputs.riemann_dt(states, dx, gamma=gamma)
    lat = lks.Lattice(25, n, n, "f32", mu=mu, dt=dt, dx=dx, bc=(1, 1), thr=thr, flag_mask=mask,
                      max_steps=steps, model="ddf", gamma=gamma, prandtl=pr, thr_qe=wl["thr_qe"])
    lat.init(rho, ux, uy, T)
    del rho, ux, uy, T
    lat.step(steps)
    torch.cuda.synchronize()
    assert lat.check() == 0
    r, u, v, t = lat.moments()
    # where the quadrant interfaces (x, y = 1/2) meet each other and the
    # outflow boundaries, the last rows included (uniform corners carry no
    # non-equilibrium to compare)
    for (x0, y0) in ((n // 2 - P // 2, n // 2 - P // 2), (0, n // 2 - 3), (n // 2 - 3, n - P)):
        R = 2 * steps + 2
        wx0, wy0 = max(x0 - R, 0), max(y0 - R, 0)
        wx1, wy1 = min(x0 + P + R, n), min(y0 + P + R, n)
        f = inputs.riemann_quadrants(n, seed=0, window=(wx0, wy0, wx1 - wx0, wy1 - wy0))
        out = orc.ddf_run(orc.ddf_equilibrium(*f[:4], gamma), steps, mu, dt, dx, bc=(1, 1),
                          gamma=gamma, prandtl=pr, thr=thr5, mask=mask)
        sl = (slice(y0 - wy0, y0 - wy0 + P), slice(x0 - wx0, x0 - wx0 + P))
        m = orc.ddf_moments(out["f"], gamma)[(slice(None),) + sl]
        e_rho = np.abs(_dpatch(r, y0, x0) - m[0]).max()
        e_u = np.hypot(_dpatch(u, y0, x0) - m[1], _dpatch(v, y0, x0) - m[2]).max() / np.hypot(m[1], m[2]).max()
        e_T = np.abs(_dpatch(t, y0, x0) - m[3]).max() / m[3].max()
        sens = out["sens"][(slice(None),) + sl]
        es = [np.abs(_dpatch(lat.sensors[k], y0, x0) - sens[k]).max() / max(np.abs(sens[k]).max(), 1e-30)
              for k in range(5)]
        print(f"patch ({x0},{y0}): rho {e_rho:.2e} u {e_u:.2e} T {e_T:.2e} sensors "
              + " ".join(f"{e:.2e}" for e in es), flush=True)
        assert e_rho <= 1e-5 and e_u <= 1e-5 and e_T <= 1e-5
        assert max(es) <= 1e-3
        bad, excl = flags_outside_band(_dpatch(lat.flags, y0, x0), out["flags"][sl], sens, thr5,
                                       mask, [max(e, 1e-6) for e in es])
        assert bad == 0, (bad, excl)
