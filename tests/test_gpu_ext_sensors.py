"""GPU parity of the extension sensors (the rest of Table I on the f
distribution, computed in the fused step) against the FP64 oracle, through
the C ABI.

Bars: FP64 storage <= 1e-11 max-normwise (kernel logic), except the two
sensors whose oracle form is the literal difference of O(1) H values (relative
H and H dissipation: the oracle's own round-off is ~1e-16 absolute, so <= 1e-8
against values ~1e-7); FP32 storage, one step from a shared FP32 state: the
bars in FP32_BARS, each a few times the measured FP32 floor of that sensor;
flags bit-exact outside the threshold band; switching the extension on changes
neither the populations nor the base sensors (bit for bit).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2603_13618_amd import inputs, lks

from gpu_util import deviation, maxnorm, to_f64

pytestmark = pytest.mark.gpu

EXT9 = ("kn", "hr", "sigma_h", "sigma_hkl", "alpha", "shear", "qh", "comp", "strain")
EXT25 = ("kn", "hr", "sigma_h", "sigma_hkl", "alpha", "shear", "qh", "qf")
LITERAL_H = ("hr", "sigma_h")
# FP32, one step from a shared state: f^neq = d - d^eq carries ~1e-7 of the
# largest deviation; the sums whose leading terms cancel by conservation (the
# relative H and the H dissipation) and the ratios of the entropic estimate
# lose a further one to two digits.  Measured (D2Q9 256^2 / D2Q25 128^2
# Riemann): kn 5.5e-7 / 4.5e-6, hr 1.4e-5 / 1.5e-4, sigma_h 6.9e-6 / 7.5e-5,
# sigma_hkl 6.7e-7 / 1.2e-6, alpha 1.9e-6 / 2.2e-5, shear 3.4e-7 / 1.2e-6,
# qh 1.4e-6 / 1.3e-5, qf - / 3.1e-6, comp 1.4e-6, strain 6.8e-7; the bars are
# about four times the larger of the two.
FP32_BARS = {"kn": 2e-5, "hr": 6e-4, "sigma_h": 3e-4, "sigma_hkl": 5e-6, "alpha": 1e-4,
             "shear": 5e-6, "qh": 5e-5, "qf": 1.5e-5, "comp": 6e-6, "strain": 3e-6}


def _oracle_ext_d2q9(f0, steps, tau):
    """Oracle extension sensors of the pre-collision state of step `steps`."""
    f = oracle.run(9, f0, steps - 1, tau=tau)["f"] if steps > 1 else f0
    g = oracle.d2q9_step(f, tau)["g"]
    return oracle.ext_sensors(9, g, tau)


def _thr_from(ref, names, lo=0.5, hi=0.9):
    """Thresholds at two quantiles of each reference sensor (so that every
    flag level occurs)."""
    t = np.full((lks.MAX_EXT, 2), np.inf)
    for name in names:
        k = lks.EXT_NAMES.index(name)
        v = ref[k][np.isfinite(ref[k])]
        t[k] = np.quantile(v, [lo, hi])
    return t


def _flags_ref(ref, names, thr):
    level = np.zeros(ref.shape[1:], np.uint8)
    for name in names:
        k = lks.EXT_NAMES.index(name)
        l = (ref[k] > thr[k, 0]).astype(np.uint8) + (ref[k] > thr[k, 1]).astype(np.uint8)
        level = np.maximum(level, l)
    return level


def _near_band(ref, names, thr, tol):
    near = np.zeros(ref.shape[1:], bool)
    for name in names:
        k = lks.EXT_NAMES.index(name)
        band = tol * np.abs(ref[k][np.isfinite(ref[k])]).max()
        for t in thr[k]:
            near |= np.abs(ref[k] - t) <= band
    return near


@pytest.mark.parametrize("n,ny,steps", [(128, 128, 30), (100, 37, 5), (6, 5, 3)])
def test_d2q9_fp64_matches_oracle(n, ny, steps):
    rho, ux, uy = inputs.smooth_random(max(n, ny, 16), seed=4, cutoff=4)
    rho, ux, uy = rho[:ny, :n], 3 * ux[:ny, :n], 3 * uy[:ny, :n]
    tau = 0.6
    f0 = oracle.equilibrium(9, rho, ux, uy)
    ref = _oracle_ext_d2q9(f0, steps, tau)
    names = ("kn", "shear", "alpha")
    thr = _thr_from(ref, names)
    flag_mask = sum(lks.flag_x(k) for k in names)
    lat = lks.Lattice(9, n, ny, "f64", tau=tau, ext=EXT9, thr_ext=thr, flag_mask=flag_mask)
    lat.init(rho, ux, uy)
    lat.step(steps)
    torch.cuda.synchronize()
    for name in EXT9:
        k = lks.EXT_NAMES.index(name)
        err = maxnorm(lat.ext(name), ref[k])
        print(name, f"{err:.2e}", flush=True)
        assert err <= (1e-8 if name in LITERAL_H else 1e-11), name
    near = _near_band(ref, names, thr, 1e-9)
    bad = (to_f64(lat.flags) != _flags_ref(ref, names, thr)) & ~near
    assert int(bad.sum()) == 0


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_extension_changes_nothing_else(dtype):
    n = 256
    rho, ux, uy = inputs.smooth_random(n, seed=2, cutoff=16)
    thr = np.array([[1e-9, 1e-8], [1e-4, 5e-4], [1e-4, 5e-4], [np.inf, np.inf]])
    # the same launch shape (the FP64 sums are reproducible per shape)
    a = lks.Lattice(9, n, n, dtype, tau=0.52, thr=thr, flag_mask=7, max_steps=8, launch_vec=2)
    b = lks.Lattice(9, n, n, dtype, tau=0.52, thr=thr, flag_mask=7, max_steps=8, launch_vec=2,
                    ext=EXT9)
    for lat in (a, b):
        lat.init(rho, ux, uy)
        lat.step(8)
    torch.cuda.synchronize()
    assert torch.equal(a.state, b.state)
    assert torch.equal(a.sensors, b.sensors[:3])
    assert torch.equal(a.flags, b.flags)
    assert torch.equal(a.sums, b.sums)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n,ny", [(96, 96), (90, 84)])     # whole tiles, ragged
def test_d2q25_extension_changes_nothing_else(dtype, n, ny):
    rho, ux, uy, T, states = inputs.riemann_quadrants(n, ny, seed=1)
    dx = 1.0 / n
    dt = inputs.riemann_dt(states, dx)
    kw = dict(mu=1e-3, dt=dt, dx=dx, bc=(1, 1), max_steps=6, flag_mask=15,
              thr=np.array([[1e-7, 1e-6], [1e-4, 1e-3], [1e-3, 1e-2], [1e-3, 1e-2]]))
    a = lks.Lattice(25, n, ny, dtype, **kw)
    b = lks.Lattice(25, n, ny, dtype, ext=EXT25, **kw)
    for lat in (a, b):
        lat.init(rho, ux, uy, T)
        lat.step(6)
    torch.cuda.synchronize()
    assert torch.equal(a.state, b.state)
    assert torch.equal(a.sensors, b.sensors[:4])
    assert torch.equal(a.flags, b.flags)
    assert torch.equal(a.sums, b.sums)


def test_d2q9_fp32_single_step_from_shared_state():
    n = 256
    rho, ux, uy = inputs.smooth_random(n, seed=5, cutoff=16)
    f = oracle.run(9, oracle.equilibrium(9, rho, ux, uy), 20, tau=0.52)["f"]
    d32 = deviation(f, 9).astype(np.float32)
    _, _, w = oracle.lattice(9)
    shared = w[:, None, None] + d32.astype(np.float64)
    g = oracle.d2q9_step(shared, 0.52)["g"]
    ref = oracle.ext_sensors(9, g, 0.52)
    lat = lks.Lattice(9, n, n, "f32", tau=0.52, ext=EXT9)
    lat.restore(torch.from_numpy(d32))
    lat.step(1)
    torch.cuda.synchronize()
    errs = {}
    for name in EXT9:
        errs[name] = maxnorm(lat.ext(name), ref[lks.EXT_NAMES.index(name)])
    print(" ".join(f"{k} {v:.2e}" for k, v in errs.items()), flush=True)
    for name, e in errs.items():
        assert e <= FP32_BARS[name], name


@pytest.mark.parametrize("nx,ny,bc", [(96, 80, (1, 1)), (40, 36, (0, 0)), (5, 3, (0, 1))])
def test_d2q25_fp64_matches_oracle(nx, ny, bc):
    rho, ux, uy, T, states = inputs.riemann_quadrants(nx, ny, seed=0)
    dx = 1.0 / max(nx, 64)
    dt = inputs.riemann_dt(states, dx)
    mu, steps = 1e-3, 8
    f0 = oracle.equilibrium(25, rho, ux, uy, T)
    f = oracle.run(25, f0, steps - 1, mu=mu, dt=dt, dx=dx, bc=bc)["f"]
    ref = oracle.ext_sensors(25, f, mu)
    names = ("qf", "sigma_hkl")
    thr = _thr_from(ref, names)
    flag_mask = sum(lks.flag_x(k) for k in names)
    lat = lks.Lattice(25, nx, ny, "f64", mu=mu, dt=dt, dx=dx, bc=bc, ext=EXT25, thr_ext=thr,
                      flag_mask=flag_mask, max_steps=steps)
    lat.init(rho, ux, uy, T)
    lat.step(steps)
    torch.cuda.synchronize()
    for name in EXT25:
        k = lks.EXT_NAMES.index(name)
        if np.abs(ref[k]).max() == 0:
            continue
        err = maxnorm(lat.ext(name), ref[k])
        print(name, f"{err:.2e}", flush=True)
        assert err <= (1e-8 if name in LITERAL_H else 1e-11), name
    near = _near_band(ref, names, thr, 1e-9)
    bad = (to_f64(lat.flags) != _flags_ref(ref, names, thr)) & ~near
    assert int(bad.sum()) == 0


def test_d2q25_fp32_single_step_from_shared_state():
    n = 128
    rho, ux, uy, T, states = inputs.riemann_quadrants(n, n, seed=2)
    dx = 1.0 / n
    dt = inputs.riemann_dt(states, dx)
    mu = 1e-3
    f = oracle.run(25, oracle.equilibrium(25, rho, ux, uy, T), 10, mu=mu, dt=dt, dx=dx,
                   bc=(1, 1))["f"]
    d32 = deviation(f, 25).astype(np.float32)
    _, _, w = oracle.lattice(25)
    ref = oracle.ext_sensors(25, w[:, None, None] + d32.astype(np.float64), mu)
    lat = lks.Lattice(25, n, n, "f32", mu=mu, dt=dt, dx=dx, bc=(1, 1), ext=EXT25)
    lat.restore(torch.from_numpy(d32))
    lat.step(1)
    torch.cuda.synchronize()
    errs = {name: maxnorm(lat.ext(name), ref[lks.EXT_NAMES.index(name)]) for name in EXT25}
    print(" ".join(f"{k} {v:.2e}" for k, v in errs.items()), flush=True)
    for name, e in errs.items():
        assert e <= FP32_BARS[name], name


def test_fault_cells_and_api_limits():
    n = 16
    rho, ux, uy = inputs.random_state((n, n), seed=3, umax=0.05)
    lat = lks.Lattice(9, n, n, "f32", tau=0.6, ext=EXT9)
    lat.init(rho, ux, uy)
    s = lat.state.clone()
    s[4, 7, 9] = -2.0                       # the rest population of one cell negative
    lat.restore(s)
    lat.step(1)
    torch.cuda.synchronize()
    for name in ("kn", "hr", "sigma_h", "sigma_hkl", "alpha"):
        v = lat.ext(name)
        assert torch.isinf(v[7, 9]) and int(torch.isinf(v).sum()) == 1, name
    assert torch.isfinite(lat.ext("shear")).all()
    with pytest.raises(lks.LksError) as e:
        lks.Lattice(9, n, n, "bf16", tau=0.6, ext=["kn"])
    assert e.value.status == 6
    with pytest.raises(lks.LksError) as e:
        lat.step(1, fused=False)
    assert e.value.status == 6
