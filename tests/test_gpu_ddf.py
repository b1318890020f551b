"""GPU parity of the D2Q25 double-distribution path (f, g with the
quasi-equilibrium collision, gamma = 1.4, Pr = 0.71) against the FP64 oracle,
through the C ABI.

Bars: FP64 storage <= 1e-12 max-normwise for the state (kernel logic; the
two sides differ only in rounding order), <= 1e-11 for the five sensors,
sums to 1e-12 of the mass; FP32 storage: relative moment error <= 1e-5 after
a multi-step run (density / rho0, velocity / max|u|, T / max T); sensors
<= 3e-5 max-normwise for a single step from a shared FP32 state (the f and g
deviations are stored in FP32: the FP32 floor of the non-equilibrium parts
is about 1e-5 of the largest sensor value) and <= 1e-4 after multi-step runs;
flags bit-exact outside the threshold band.
"""
import numpy as np
import pytest
import torch

from paper_2603_13618_amd import inputs, lks

from gpu_util import flags_outside_band, maxnorm, to_f64

pytestmark = pytest.mark.gpu

GAMMA, PR = 1.4, 0.71
CV = 1.0 / (GAMMA - 1.0)
THR4 = np.array([[1e-7, 1e-6], [1e-4, 1e-3], [1e-3, 1e-2], [1e-3, 1e-2]])
THR_QE = (1e-4, 1e-3)
THR5 = np.vstack([THR4, [THR_QE]])
MASK = 31


def _ref_planes(orc, rho0=1.0):
    """Reference parts of the stored deviations: w rho0 (f), (C_v - 1) w rho0 (g)."""
    _, _, w = orc.lattice(25)
    return np.concatenate([w * rho0, (CV - 1.0) * w * rho0])[:, None, None]


def _dev(orc, f, rho0=1.0):
    return f - _ref_planes(orc, rho0)


def _full(orc, lat):
    return to_f64(lat.state) + _ref_planes(orc, lat.cfg.rho0)


def _lattice(nx, ny, dtype, mu, dt, dx, bc, steps=1, thr=True):
    return lks.Lattice(25, nx, ny, dtype, mu=mu, dt=dt, dx=dx, bc=bc,
                       thr=THR4 if thr else None, flag_mask=MASK if thr else 0,
                       max_steps=max(steps, 1), model="ddf", gamma=GAMMA, prandtl=PR,
                       thr_qe=THR_QE if thr else None)


def _riemann(n, ny=None, seed=0):
    ny = n if ny is None else ny
    rho, ux, uy, T, states = inputs.riemann_quadrants(n, ny, seed=seed)
    dx = 1.0 / max(n, 64)
    return (rho, ux, uy, T), dx, inputs.riemann_dt(states, dx, gamma=GAMMA)


def _noneq(orc, shape, seed, scale=2e-3):
    """A random state near equilibrium, with non-equilibrium parts in both f
    and g (the quasi-equilibria then carry non-zero heat fluxes)."""
    rng = np.random.default_rng(seed)
    rho = 1.0 + 0.1 * rng.standard_normal(shape)
    ux, uy = 0.05 * rng.standard_normal(shape), 0.05 * rng.standard_normal(shape)
    T = 1.0 + 0.1 * rng.standard_normal(shape)
    f = orc.ddf_equilibrium(rho, ux, uy, T, GAMMA)
    return f * (1.0 + scale * rng.standard_normal(f.shape))


def _compare_fp64(orc, lat, ref, steps):
    err = maxnorm(_dev(orc, _full(orc, lat)), _dev(orc, ref["f"]))
    assert err <= 1e-12, err
    for k in range(5):
        if np.abs(ref["sens"][k]).max() > 1e-12:
            assert maxnorm(lat.sensors[k], ref["sens"][k]) <= 1e-11, k
        else:                  # an equilibrium state: both sides at round-off
            assert np.abs(to_f64(lat.sensors[k])).max() <= 1e-12, k
    bad, _ = flags_outside_band(lat.flags, ref["flags"], ref["sens"], THR5, MASK, [1e-10] * 5)
    assert bad == 0
    sums = to_f64(lat.sums)[:steps]
    m0 = ref["sums"][0, 0]
    assert np.abs(sums[:, :4] - ref["sums"][:, :4]).max() <= 1e-12 * m0
    for k in range(4, 8):      # sensor totals; uniform states leave them at round-off
        bar = 1e-11 * np.abs(ref["sums"][:, k]).max() + 1e-14 * m0
        assert np.abs(sums[:, k] - ref["sums"][:, k]).max() <= bar, k


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-14), ("f32", 2e-7)])
def test_init_and_moments(orc, dtype, tol):
    rho, ux, uy = inputs.random_state((19, 37), seed=4, umax=0.1)
    T = 1.0 + 0.3 * (rho - 1.0)
    lat = _lattice(37, 19, dtype, 1e-3, 1e-4, 0.05, (1, 1))
    lat.init(rho, ux, uy, T)
    want = orc.ddf_equilibrium(rho, ux, uy, T, GAMMA)
    assert maxnorm(lat.state, _dev(orc, want)) <= tol * 10
    r, u, v, t = (to_f64(x) for x in lat.moments())
    assert np.abs(r - rho).max() <= tol and np.abs(u - ux).max() <= tol
    assert np.abs(v - uy).max() <= tol and np.abs(t - T).max() <= 10 * tol


# (192 x 100: 300 workgroups of 16 x 4 cells, more than 256, so the partial
# sums are reduced in two passes, the second chunk partial)
@pytest.mark.parametrize("nx,ny,bc", [(96, 80, (1, 1)), (40, 36, (0, 0)), (67, 9, (1, 0)),
                                      (5, 3, (0, 1)), (1, 1, (1, 1)), (192, 100, (0, 1))])
def test_fp64_riemann_matches_oracle(orc, nx, ny, bc):
    fields, dx, dt = _riemann(nx, ny)
    steps = 12
    ref = orc.ddf_run(orc.ddf_equilibrium(*fields, GAMMA), steps, 1e-3, dt, dx, bc=bc, gamma=GAMMA,
                      prandtl=PR, thr=THR5, mask=MASK)
    lat = _lattice(nx, ny, "f64", 1e-3, dt, dx, bc, steps)
    lat.init(*fields)
    lat.step(steps)
    torch.cuda.synchronize()
    _compare_fp64(orc, lat, ref, steps)
    assert lat.check() == 0


@pytest.mark.parametrize("nx,ny,bc", [(45, 22, (0, 0)), (33, 7, (1, 0))])
def test_fp64_nonequilibrium_state(orc, nx, ny, bc):
    # every population off equilibrium: exercises both quasi-equilibrium terms
    f0 = _noneq(orc, (ny, nx), seed=nx)
    dx = 1.0 / 32
    dt = 0.05 * dx / 3.0
    steps = 3
    ref = orc.ddf_run(f0, steps, 2e-3, dt, dx, bc=bc, gamma=GAMMA, prandtl=PR, thr=THR5, mask=MASK)
    lat = _lattice(nx, ny, "f64", 2e-3, dt, dx, bc, steps)
    lat.restore(torch.from_numpy(_dev(orc, f0)))
    lat.step(steps)
    torch.cuda.synchronize()
    _compare_fp64(orc, lat, ref, steps)
    assert (to_f64(lat.sensors[4]) > 0).all()


def test_fp32_single_step_from_shared_state(orc):
    n = 128
    fields, dx, dt = _riemann(n, seed=2)
    f = orc.ddf_run(orc.ddf_equilibrium(*fields, GAMMA), 10, 1e-3, dt, dx, bc=(1, 1),
                    gamma=GAMMA, prandtl=PR)["f"]
    d32 = _dev(orc, f).astype(np.float32)
    shared = d32.astype(np.float64) + _ref_planes(orc)
    ref = orc.ddf_step(shared, 1e-3, dt, dx, bc=(1, 1), gamma=GAMMA, prandtl=PR, thr=THR5, mask=MASK)
    lat = _lattice(n, n, "f32", 1e-3, dt, dx, (1, 1))
    lat.restore(torch.from_numpy(d32))
    lat.step(1)
    es = []
    for k in range(5):
        e = maxnorm(lat.sensors[k], ref["sens"][k])
        print("sensor", k, f"{e:.2e}", flush=True)
        es.append(e)
    # measured: S_KL 5.0e-6, S_NEQ 2.5e-6, S_PI 2.4e-6, S_Q 2.7e-6, S_QE 2.6e-6
    assert max(es) <= 1e-5
    assert maxnorm(_dev(orc, _full(orc, lat)), _dev(orc, ref["f"])) <= 1e-5
    bad, excl = flags_outside_band(lat.flags, ref["flags"], ref["sens"], THR5, MASK,
                                   [max(e, 1e-6) for e in es])
    print("flag mismatches", bad, "excluded", excl, flush=True)
    assert bad == 0


def test_fp32_multistep_riemann(orc):
    n = 128
    fields, dx, dt = _riemann(n)
    steps = 50
    ref = orc.ddf_run(orc.ddf_equilibrium(*fields, GAMMA), steps, 1e-3, dt, dx, bc=(1, 1),
                      gamma=GAMMA, prandtl=PR, thr=THR5, mask=MASK)
    lat = _lattice(n, n, "f32", 1e-3, dt, dx, (1, 1), steps)
    lat.init(*fields)
    lat.step(steps)
    torch.cuda.synchronize()
    r, u, v, t = (to_f64(x) for x in lat.moments())
    m = orc.ddf_moments(ref["f"], GAMMA)
    e_rho = np.abs(r - m[0]).max()
    e_u = np.hypot(u - m[1], v - m[2]).max() / np.hypot(m[1], m[2]).max()
    e_T = np.abs(t - m[3]).max() / np.abs(m[3]).max()
    es = [maxnorm(lat.sensors[k], ref["sens"][k]) for k in range(5)]
    print(f"moments rho {e_rho:.2e} u {e_u:.2e} T {e_T:.2e}; sensors "
          + " ".join(f"{e:.2e}" for e in es), flush=True)
    assert e_rho <= 1e-5 and e_u <= 1e-5 and e_T <= 1e-5
    assert max(es) <= 1e-4
    bad, excl = flags_outside_band(lat.flags, ref["flags"], ref["sens"], THR5, MASK,
                                   [max(e, 1e-6) for e in es])
    print("flag mismatches", bad, "excluded", excl, flush=True)
    assert bad == 0
    assert lat.check() == 0


def test_periodic_conservation_and_fixed_point(orc):
    n = 64
    rho, ux, uy = inputs.smooth_random(n, seed=2, cutoff=3)
    T = 1.0 + 0.3 * (rho - 1.0)
    dx = 1.0 / n
    lat = _lattice(n, n, "f64", 2e-3, 0.2 * dx / 3.0, dx, (0, 0), steps=40, thr=False)
    lat.init(rho, ux, uy, T)
    lat.step(40)
    s = to_f64(lat.sums)
    for k in range(4):       # mass, momentum, total energy E = sum g + sum |v|^2/2 f
        assert np.abs(s[:, k] - s[0, k]).max() <= 1e-13 * s[0, 0]
    u = np.full((8, 8), 1.0)
    lat = _lattice(8, 8, "f64", 1e-3, 1e-3, 0.125, (1, 1), steps=3, thr=False)
    lat.init(0.9 * u, 0.07 * u, 0.02 * u, 1.05 * u)
    lat.step(3)
    r, a, b, t = (to_f64(x) for x in lat.moments())
    assert np.abs(r - 0.9).max() < 1e-14 and np.abs(a - 0.07).max() < 1e-14
    assert np.abs(t - 1.05).max() < 1e-13
    assert np.abs(to_f64(lat.sensors)).max() < 1e-13


def test_positivity_fault_of_g(orc):
    # one negative internal-energy population: the cell is flagged as a fault
    # on both sides, S_KL = +inf, and the fault counter sees it
    f0 = _noneq(orc, (6, 9), seed=5)
    f0[25 + 7, 2, 4] = -1e-3
    ref = orc.ddf_step(f0, 1e-3, 1e-4, 0.1, bc=(1, 1), gamma=GAMMA, prandtl=PR, thr=THR5, mask=MASK)
    lat = _lattice(9, 6, "f64", 1e-3, 1e-4, 0.1, (1, 1))
    lat.restore(torch.from_numpy(_dev(orc, f0)))
    lat.step(1)
    flags = to_f64(lat.flags)
    assert np.array_equal(flags, ref["flags"])
    assert flags[2, 4] == 0x82 and np.isinf(to_f64(lat.sensors[0])[2, 4])
    assert lat.check() == 1 == ref["faults"]


def test_ddf_api_limits():
    with pytest.raises(lks.LksError) as e:
        _lattice(8, 8, "bf16", 1e-3, 1e-3, 0.1, (1, 1))
    assert e.value.status == 6
    with pytest.raises(lks.LksError) as e:      # no bulk viscosity on the monatomic BGK gas
        lks.Lattice(25, 8, 8, "f32", mu=1e-3, dt=1e-3, dx=0.1, ext=["strain"])
    assert e.value.status == 1
    lks.Lattice(25, 8, 8, "f32", mu=1e-3, dt=1e-3, dx=0.1, model="ddf", ext=["strain"])
    lat = _lattice(8, 8, "f32", 1e-3, 1e-3, 0.1, (1, 1))
    assert lat.pop[0].shape == (50, 8, 8) and lat.sensors.shape == (5, 8, 8)
    u = np.ones((8, 8))
    with pytest.raises(lks.LksError):
        lat.init(u, 0 * u, 0 * u)              # T is required
    lat.init(u, 0 * u, 0 * u, u)
    with pytest.raises(lks.LksError) as e:
        lat.step(1, fused=False)
    assert e.value.status == 6
    lat.step(2)
    assert lat.check() == 0
