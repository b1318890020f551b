"""GPU parity of the extension sensors on the double distribution (the rest
of Table I with the g terms superposed and the quasi-equilibrium collision as
Omega) against the FP64 oracle, through the C ABI.

Bars: FP64 storage <= 1e-11 max-normwise, except the relative H and the H
dissipation, whose oracle form is the literal difference of O(1) H values
(<= 1e-8, as for the single distribution); FP32 storage, one step from a
shared FP32 state: each sensor within a few times its measured FP32 floor
(FP32_BARS); flags of extension sensors bit-exact outside the threshold band;
switching the extension on changes neither the state nor the base sensors
(bit for bit).  Compression and strain take the model's second viscosity
-(gamma - 1) mu (Sec. II.A.2, eq. visc_bluk_1).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2603_13618_amd import inputs, lks

from gpu_util import maxnorm, to_f64

pytestmark = pytest.mark.gpu

GAMMA, PR = 1.4, 0.71
CV = 1.0 / (GAMMA - 1.0)
EXT = ("kn", "hr", "sigma_h", "sigma_hkl", "alpha", "shear", "qh", "qf", "comp", "strain")
LITERAL_H = ("hr", "sigma_h")
# FP32 floors measured on a 128^2 Riemann state, one step from a shared FP32
# state: kn 1.6e-6, hr 7.9e-6, sigma_h 1.9e-6, sigma_hkl 2.0e-6, alpha 4.6e-6,
# shear 9.3e-7, qh 2.5e-6, qf 2.5e-6, comp 7.0e-6, strain 6.9e-6 (both built
# on tr P, a sum of two stress components that largely cancel where the flow
# shears); the bars are about four times them
FP32_BARS = {"kn": 7e-6, "hr": 3e-5, "sigma_h": 8e-6, "sigma_hkl": 8e-6, "alpha": 2e-5,
             "shear": 4e-6, "qh": 1e-5, "qf": 1e-5, "comp": 3e-5, "strain": 3e-5}


def _ref_planes(rho0=1.0):
    _, _, w = oracle.lattice(25)
    return np.concatenate([w * rho0, (CV - 1.0) * w * rho0])[:, None, None]


def _lat(nx, ny, dtype, mu, dt, dx, bc, ext=EXT, thr_ext=None, flag_mask=0):
    return lks.Lattice(25, nx, ny, dtype, mu=mu, dt=dt, dx=dx, bc=bc, model="ddf", gamma=GAMMA,
                       prandtl=PR, ext=ext, thr_ext=thr_ext, flag_mask=flag_mask)


def _riemann_state(n, steps, mu, seed=0):
    rho, ux, uy, T, states = inputs.riemann_quadrants(n, seed=seed)
    dx = 1.0 / max(n, 64)
    dt = inputs.riemann_dt(states, dx, gamma=GAMMA)
    f = oracle.ddf_run(oracle.ddf_equilibrium(rho, ux, uy, T, GAMMA), steps, mu, dt, dx, bc=(1, 1),
                       gamma=GAMMA, prandtl=PR)["f"]
    return f, dt, dx


def _noneq(shape, seed, scale=2e-3):
    rng = np.random.default_rng(seed)
    rho = 1.0 + 0.1 * rng.standard_normal(shape)
    ux, uy = 0.05 * rng.standard_normal(shape), 0.05 * rng.standard_normal(shape)
    T = 1.0 + 0.1 * rng.standard_normal(shape)
    f = oracle.ddf_equilibrium(rho, ux, uy, T, GAMMA)
    return f * (1.0 + scale * rng.standard_normal(f.shape))


@pytest.mark.parametrize("case", ["noneq-45x22", "noneq-7x5", "riemann-96"])
def test_fp64_matches_oracle(case):
    mu = 2e-3
    if case.startswith("noneq"):
        nx, ny = (45, 22) if case.endswith("45x22") else (7, 5)
        f0, dt, dx = _noneq((ny, nx), seed=nx), 0.05 / 32 / 3.0, 1.0 / 32
    else:
        f0, dt, dx = _riemann_state(96, 10, mu)
        ny, nx = f0.shape[1:]
    lat = _lat(nx, ny, "f64", mu, dt, dx, (1, 1))
    lat.restore(torch.from_numpy(f0 - _ref_planes()))
    lat.step(1)
    ref = oracle.ddf_ext_sensors(f0, mu, GAMMA, PR)
    for name in EXT:
        k = lks.EXT_NAMES.index(name)
        e = maxnorm(lat.ext(name), ref[k])
        print(case, name, f"{e:.2e}", flush=True)
        assert e <= (1e-8 if name in LITERAL_H else 1e-11), name


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n,ny", [(64, 64), (60, 50)])     # whole tiles, ragged
def test_base_outputs_unchanged_by_the_extension(dtype, n, ny):
    f0, dt, dx = _riemann_state(64, 5, 1e-3)
    d = torch.from_numpy(np.ascontiguousarray(f0[:, :ny, :n]) - _ref_planes())
    outs = []
    for ext in (None, EXT):
        lat = _lat(n, ny, dtype, 1e-3, dt, dx, (1, 1), ext=ext)
        lat.restore(d)
        lat.step(2)
        torch.cuda.synchronize()
        outs.append((lat.state.clone(), lat.sensors[:5].clone(), lat.flags.clone()))
    for name, a, b in zip(("state", "sensors", "flags"), *outs):
        if not torch.equal(a, b):
            diff = (a.double() - b.double()).abs()
            print(name, "differs at", int((diff > 0).sum()), "of", diff.numel(), "max", float(diff.max()),
                  "planes", sorted(set(torch.nonzero(diff.reshape(diff.shape[0], -1).amax(1) > 0).flatten().tolist()))
                  if diff.dim() == 3 else "-", flush=True)
    for a, b in zip(*outs):
        assert torch.equal(a, b)


def test_fp32_single_step_from_shared_state():
    mu = 1e-3
    f, dt, dx = _riemann_state(128, 10, mu, seed=2)
    d32 = (f - _ref_planes()).astype(np.float32)
    shared = d32.astype(np.float64) + _ref_planes()
    ref = oracle.ddf_ext_sensors(shared, mu, GAMMA, PR)
    lat = _lat(128, 128, "f32", mu, dt, dx, (1, 1))
    lat.restore(torch.from_numpy(d32))
    lat.step(1)
    bad = []
    for name in EXT:
        e = maxnorm(lat.ext(name), ref[lks.EXT_NAMES.index(name)])
        print("fp32", name, f"{e:.2e}", "bar", FP32_BARS[name], flush=True)
        if not e <= FP32_BARS[name]:
            bad.append(name)
    assert not bad


def test_flags_of_extension_sensors():
    mu = 2e-3
    f0 = _noneq((24, 40), seed=3, scale=5e-3)
    ref = oracle.ddf_ext_sensors(f0, mu, GAMMA, PR)
    names = ("kn", "sigma_hkl", "qf")
    thr = np.full((lks.MAX_EXT, 2), np.inf)
    mask = 0
    for name in names:
        k = lks.EXT_NAMES.index(name)
        thr[k] = np.quantile(ref[k], [0.5, 0.9])
        mask |= lks.flag_x(name)
    lat = _lat(40, 24, "f64", mu, 0.05 / 32 / 3.0, 1.0 / 32, (0, 0), thr_ext=thr, flag_mask=mask)
    lat.restore(torch.from_numpy(f0 - _ref_planes()))
    lat.step(1)
    level = np.zeros(ref.shape[1:], np.uint8)
    near = np.zeros(ref.shape[1:], bool)
    for name in names:
        k = lks.EXT_NAMES.index(name)
        level = np.maximum(level, (ref[k] > thr[k, 0]).astype(np.uint8) + (ref[k] > thr[k, 1]))
        for t in thr[k]:
            near |= np.abs(ref[k] - t) <= 1e-9 * np.abs(ref[k]).max()
    got = to_f64(lat.flags)
    assert (got[~near] == level[~near]).all()
    assert (level == 2).any() and (level == 0).any()


def test_ddf_extension_limits():
    # compression and strain exist on the double distribution, not on the
    # monatomic single distribution
    with pytest.raises(lks.LksError):
        lks.Lattice(25, 8, 8, "f32", mu=1e-3, dt=1e-3, dx=0.1, ext=["comp"])
    assert _lat(8, 8, "f32", 1e-3, 1e-3, 0.1, (1, 1), ext=["comp", "strain"]).sensors.shape == (7, 8, 8)
    lat = _lat(8, 8, "f32", 1e-3, 1e-3, 0.1, (1, 1), ext=["kn", "qf"])
    assert lat.sensors.shape == (7, 8, 8)
    assert lat.ext("qf").data_ptr() == lat.sensors[6].data_ptr()
