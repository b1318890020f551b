"""GPU macroscopic class-1 sensors (central differences) against the oracle,
and the paper's class-1 validation on the GPU: kinetic sensors from the
populations against macroscopic ones from the moments of the same state
(Sec. IV).

Bars: the device kernel vs the oracle (same formulas in FP64): 1e-12
max-normwise.  Kinetic vs macroscopic: relative L2 over the grid; they differ
by the higher-order Chapman-Enskog terms, the central-difference error and,
on D2Q25, the explicit time step (dt/tau = 0.15).  The FP64 oracle gives
1.4-2.8 % (D2Q9, 128^2, tau = 0.8, 20 steps) and 1.6-2.3 % for the rates and
q_H, 3-5 % for q_F (D2Q25, 96^2, 200 steps); bars 5 % and 6 % (q_F).
"""
import numpy as np
import pytest
import torch

from oracle import macro
from paper_2603_13618_amd import inputs, lks

from gpu_util import maxnorm, to_f64

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.mark.parametrize("q,nx,ny,bc,per_rho", [(9, 70, 37, (0, 0), True), (25, 64, 64, (1, 1), False),
                                                (25, 45, 19, (0, 1), True), (25, 5, 3, (1, 0), False),
                                                (9, 1, 1, (0, 0), False)])
def test_macro_matches_oracle(q, nx, ny, bc, per_rho):
    rng = np.random.default_rng(nx * ny)
    fields = [1.0 + 0.1 * rng.standard_normal((ny, nx)), 0.1 * rng.standard_normal((ny, nx)),
              0.1 * rng.standard_normal((ny, nx)), 1.0 + 0.1 * rng.standard_normal((ny, nx))]
    dx = 1.0 if q == 9 else 0.013
    kw = dict(tau=0.6) if q == 9 else dict(mu=1e-3, dt=1e-4, dx=dx, bc=bc)
    lat = lks.Lattice(q, nx, ny, "f64", **kw)
    got = lat.macro_sensors(*[_dev(a) for a in fields], mu=0.3, lam=-0.2, kappa=0.7, per_rho=per_rho)
    want = macro.macro_sensors(*fields, 0.3, -0.2, 0.7, dx=dx, bc=bc if q == 25 else (0, 0),
                               per_rho=per_rho)
    for name in macro.NAMES:
        w = want[name]
        if np.abs(w).max() > 0:
            assert maxnorm(got[name], w) <= 1e-12, name
        else:
            assert np.abs(to_f64(got[name])).max() == 0.0, name
    # a subset lands in consecutive planes in bit order
    sub = lat.macro_sensors(*[_dev(a) for a in fields[:3]], None, mu=0.3, which=("qh", "c"))
    assert list(sub) == ["c", "qh"]
    want_qh = macro.macro_sensors(*fields, 0.3, 0.0, 0.0, dx=dx, bc=bc if q == 25 else (0, 0),
                                  which=("qh",))["qh"]
    if np.abs(want_qh).max() > 0:
        assert maxnorm(sub["qh"], want_qh) <= 1e-12


def test_macro_api_limits():
    lat = lks.Lattice(9, 16, 16, "f64", tau=0.6)
    f = [_dev(np.ones((16, 16))) for _ in range(4)]
    out = torch.empty((7, 16, 16), dtype=torch.float64, device="cuda")
    L = lks.lib()
    import ctypes
    tr = lks.Transport(0.1, 0.0, 0.1, 0, 0)
    P = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
    assert L.lks_macro_sensors(lat.ctx, P(f[0]), P(f[1]), P(f[2]), P(f[3]), ctypes.byref(tr), 0, P(out)) == 1
    assert L.lks_macro_sensors(lat.ctx, P(f[0]), P(f[1]), P(f[2]), P(f[3]), ctypes.byref(tr), 1 << 7, P(out)) == 1
    assert L.lks_macro_sensors(lat.ctx, P(f[0]), P(f[1]), P(f[2]), None, ctypes.byref(tr), 1 << 5, P(out)) == 1
    assert L.lks_macro_sensors(lat.ctx, P(f[0]), P(f[1]), P(f[2]), P(f[3]), ctypes.byref(tr), 1, P(f[1])) == 1
    tr_rho = lks.Transport(0.1, 0.0, 0.1, 1, 0)
    assert L.lks_macro_sensors(lat.ctx, None, P(f[1]), P(f[2]), P(f[3]), ctypes.byref(tr_rho), 1, P(out)) == 1
    bad = lks.Transport(0.1, 0.0, 0.1, 0, 1)
    assert L.lks_macro_sensors(lat.ctx, P(f[0]), P(f[1]), P(f[2]), P(f[3]), ctypes.byref(bad), 1, P(out)) == 1
    assert L.lks_macro_sensors(lat.ctx, P(f[0]), P(f[1]), P(f[2]), P(f[3]), ctypes.byref(tr), 127, P(out)) == 0


def _rel(a, b):
    a, b = to_f64(a), to_f64(b)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_class1_kinetic_vs_macroscopic_d2q9():
    n, tau = 128, 0.8
    rho, ux, uy = inputs.smooth_random(n, seed=0, cutoff=4)
    lat = lks.Lattice(9, n, n, "f32", tau=tau, ext=["shear", "comp", "strain", "qh"])
    lat.init(rho, ux, uy)
    lat.step(20)
    m = lat.moments()
    mac = lat.macro_sensors(m[0], m[1], m[2], None, mu=tau / 3.0, per_rho=True,
                            which=("tau", "s", "c", "e", "qh"))
    pairs = (("shear", "s"), ("comp", "c"), ("strain", "e"), ("qh", "qh"))
    for kn, mn in pairs:
        e = _rel(lat.ext(kn), mac[mn])
        print(kn, f"{e:.3e}", flush=True)
        assert e <= 0.05, kn
    e = _rel(lat.sensors[2], mac["tau"])                   # S_PI = |P^neq| vs |tau_NS|
    print("S_PI", f"{e:.3e}", flush=True)
    assert e <= 0.05


def test_class1_kinetic_vs_macroscopic_d2q25():
    n, mu = 96, 2e-3
    dx = 1.0 / n
    rho, ux, uy = inputs.smooth_random(n, seed=1, cutoff=3)
    T = 1.0 + 3.0 * (rho - 1.0)
    ux, uy = 3.0 * ux, 3.0 * uy
    dt = inputs.cfl_dt((rho, ux, uy, T), dx, gamma=2.0, cfl=0.05)
    lat = lks.Lattice(25, n, n, "f64", mu=mu, dt=dt, dx=dx, bc=(0, 0), ext=["shear", "qh", "qf"])
    lat.init(rho, ux, uy, T)
    lat.step(200)
    m = lat.moments()                                        # the state the next step's sensors read
    m = [t.clone() for t in m]
    lat.step(1)
    mac = lat.macro_sensors(*m, mu=mu, lam=-mu, kappa=2.0 * mu, which=("s", "qh", "qf"))
    for kn, mn, bar in (("shear", "s", 0.05), ("qh", "qh", 0.05), ("qf", "qf", 0.06)):
        e = _rel(lat.ext(kn), mac[mn])
        print(kn, f"{e:.3e}", flush=True)
        assert e <= bar, kn
