"""The row-interleaved population layout ([ny][Q][nx]) against the plane-major
one ([Q][ny][nx]) and against the FP64 oracle, through the C ABI.

The layouts hold the same values at different addresses and every kernel does
the same arithmetic in the same order on both, so all outputs (state, sensors,
flags, sums, moments, adjoint gradients) must be bit-identical between them.
One FP64 D2Q9 run and one FP64 D2Q25 run are also compared with the oracle
directly, to the bars of the plane-major parity tests (state and moments
<= 1e-12, sensors <= 1e-12 on D2Q9 and <= 1e-11 on D2Q25).
"""
import ctypes

import numpy as np
import pytest
import torch

from paper_2603_13618_amd import adjoint, inputs, lks

from gpu_util import deviation, full_state, maxnorm, to_f64

pytestmark = pytest.mark.gpu


def _same(a, b, what):
    a, b = a.detach().cpu(), b.detach().cpu()
    assert a.shape == b.shape, what
    if a.dtype in (torch.bfloat16, torch.float16):
        a, b = a.view(torch.int16), b.view(torch.int16)
    ok = torch.equal(a, b) or (a.is_floating_point() and bool(((a == b) | (a.isnan() & b.isnan())).all()))
    assert ok, what


def _quantile_thr(sens, planes):
    thr = np.full((4, 2), np.inf)
    for k in range(planes):
        s = to_f64(sens[k]).ravel()
        s = s[np.isfinite(s)]
        thr[k] = np.quantile(s, [0.4, 0.8])
    return thr


def _run_pair(make, init, steps, fused=True):
    """Run the same configuration in both layouts; return the two lattices."""
    out = []
    for layout in ("planes", "rows"):
        lat = make(layout)
        init(lat)
        lat.step(steps, fused=fused)
        out.append(lat)
    torch.cuda.synchronize()
    return out


def _check_pair(a, b, nsens, same_shape=True):
    assert a.layout == lks.LAYOUT_PLANES and b.layout == lks.LAYOUT_ROWS
    # the rows context's buffers really are [ny][Q][nx]
    assert b.state.stride() == (b.nx, b.Q * b.nx, 1)
    _same(a.state, b.state, "state")
    _same(a.sensors[:nsens], b.sensors[:nsens], "sensors")
    _same(a.flags, b.flags, "flags")
    if same_shape:
        _same(a.sums, b.sums, "sums")
    else:
        # other launch shapes group the per-workgroup partial sums differently
        sa, sb = to_f64(a.sums), to_f64(b.sums)
        assert np.abs(sa - sb).max() <= 1e-14 * np.abs(sa).max()
    for k, (x, y) in enumerate(zip(a.moments(), b.moments())):
        _same(x, y, f"moment {k}")
    assert a.check() == b.check()
    # the host copy of a rows state comes back as [Q, ny, nx]
    np.testing.assert_array_equal(b.read_host(0), a.read_host(0))


D2Q9_CASES = [
    # dtype, launch_vec, fused, ext, nx, ny
    ("f32", 0, True, None, 200, 72),
    ("f32", 1, True, None, 197, 33),
    ("f32", 0, False, None, 200, 72),
    ("f64", 0, True, None, 200, 40),
    ("bf16", 0, True, None, 256, 40),
    ("f16", 1, True, None, 99, 17),
    ("f32", 0, True, ("kn", "shear", "alpha", "qh"), 200, 72),
    ("f64", 0, True, ("hr", "sigma_hkl", "strain"), 96, 24),
]


@pytest.mark.parametrize("dtype,vec,fused,ext,nx,ny", D2Q9_CASES)
def test_d2q9_layouts_bit_identical(dtype, vec, fused, ext, nx, ny):
    print("case", dtype, vec, fused, ext, nx, ny, flush=True)
    rho, ux, uy = inputs.random_state((ny, nx), seed=11, umax=0.05)
    probe = lks.Lattice(9, nx, ny, dtype, tau=0.6, launch_vec=vec, max_steps=12)
    probe.init(rho, ux, uy)
    probe.step(12)
    thr = _quantile_thr(probe.sensors, 3)
    nsens = 3 + (len(ext) if ext else 0)
    mask = lks.S_KL | lks.S_NEQ | lks.S_PI

    def make(layout, rows=2):
        return lks.Lattice(9, nx, ny, dtype, tau=0.6, thr=thr, flag_mask=mask, max_steps=16,
                           launch_vec=vec, launch_rows=rows, ext=ext, layout=layout)

    # the same launch shape in both layouts: everything bit-identical
    a, b = _run_pair(make, lambda lat: lat.init(rho, ux, uy), 12, fused=fused)
    assert int((a.flags > 0).sum()) > 0
    _check_pair(a, b, nsens)
    # each layout at its automatic launch shape: the sums may differ in rounding
    a, b = _run_pair(lambda layout: make(layout, 0), lambda lat: lat.init(rho, ux, uy), 12,
                     fused=fused)
    _check_pair(a, b, nsens, same_shape=False)


@pytest.mark.parametrize("dtype,model,ext,nx,ny,bc", [
    ("f32", "bgk", None, 50, 37, (lks.OUTFLOW, lks.OUTFLOW)),
    ("f64", "bgk", None, 40, 24, (lks.PERIODIC, lks.OUTFLOW)),
    ("f32", "bgk", ("kn", "qf", "sigma_h"), 48, 40, (lks.OUTFLOW, lks.PERIODIC)),
    ("f32", "ddf", None, 50, 37, (lks.OUTFLOW, lks.OUTFLOW)),
    ("f64", "ddf", None, 36, 20, (lks.PERIODIC, lks.PERIODIC)),
    ("f32", "ddf", ("kn", "hr", "qf"), 40, 24, (lks.OUTFLOW, lks.OUTFLOW)),
])
def test_d2q25_layouts_bit_identical(dtype, model, ext, nx, ny, bc):
    print("case", dtype, model, ext, nx, ny, bc, flush=True)
    rho, ux, uy, T, states = inputs.riemann_quadrants(nx, ny, seed=4)
    dx = 1.0 / max(nx, 64)
    dt = inputs.riemann_dt(states, dx, gamma=1.4 if model == "ddf" else 2.0)
    ddf = model == "ddf"
    kw = dict(model=model, gamma=1.4, prandtl=0.71) if ddf else {}
    probe = lks.Lattice(25, nx, ny, dtype, mu=1e-3, dt=dt, dx=dx, bc=bc, max_steps=6, **kw)
    probe.init(rho, ux, uy, T)
    probe.step(6)
    base = 5 if ddf else 4
    thr = _quantile_thr(probe.sensors, 4)
    extra = {}
    if ddf:
        s = to_f64(probe.sensors[4]).ravel()
        extra = dict(thr_qe=tuple(np.quantile(s[np.isfinite(s)], [0.4, 0.8])))
    mask = 31 if ddf else 15
    nsens = base + (len(ext) if ext else 0)

    def make(layout):
        return lks.Lattice(25, nx, ny, dtype, mu=1e-3, dt=dt, dx=dx, bc=bc, thr=thr,
                           flag_mask=mask, max_steps=8, ext=ext, layout=layout, **kw, **extra)

    a, b = _run_pair(make, lambda lat: lat.init(rho, ux, uy, T), 6)
    assert int((a.flags > 0).sum()) > 0
    _check_pair(a, b, nsens)


def test_d2q9_rows_fp64_matches_oracle(orc):
    rho, ux, uy = inputs.smooth_random(64, seed=5, cutoff=6)
    thr = np.array([[1e-9, 1e-8], [1e-5, 1e-4], [1e-5, 1e-4], [np.inf, np.inf]])
    mask = lks.S_KL | lks.S_NEQ | lks.S_PI
    ref = orc.run(9, orc.equilibrium(9, rho, ux, uy), 40, tau=0.55, thr=thr, mask=mask)
    lat = lks.Lattice(9, 64, 64, "f64", tau=0.55, thr=thr, flag_mask=mask, max_steps=40,
                      layout="rows")
    lat.init(rho, ux, uy)
    lat.step(40)
    r, u, v, _ = lat.moments()
    errs = [maxnorm(r, ref["mom"][0]), maxnorm(u, ref["mom"][1]), maxnorm(v, ref["mom"][2])]
    errs += [maxnorm(lat.sensors[k], ref["sens"][k]) for k in range(3)]
    print("errors", [f"{e:.1e}" for e in errs], flush=True)
    assert max(errs) <= 1e-12


def test_d2q25_rows_fp64_matches_oracle(orc):
    nx, ny = 40, 28
    rho, ux, uy, T, states = inputs.riemann_quadrants(nx, ny, seed=2)
    dx = 1.0 / 64
    dt = inputs.riemann_dt(states, dx)
    bc = (lks.OUTFLOW, lks.OUTFLOW)
    f0 = orc.equilibrium(25, rho, ux, uy, T)
    ref = orc.run(25, f0, 10, mu=1e-3, dt=dt, dx=dx, bc=bc)
    lat = lks.Lattice(25, nx, ny, "f64", mu=1e-3, dt=dt, dx=dx, bc=bc, max_steps=10, layout="rows")
    lat.init(rho, ux, uy, T)
    lat.step(10)
    # the oracle's moments are those of the last step's pre-collision state;
    # compare the final states themselves (deviations) and the sensors
    err = maxnorm(deviation(full_state(lat, 25), 25), deviation(ref["f"], 25))
    errs = [maxnorm(lat.sensors[k], ref["sens"][k]) for k in range(4)]
    print("state", f"{err:.1e}", "sensors", [f"{e:.1e}" for e in errs], flush=True)
    assert err <= 1e-12 and max(errs) <= 1e-11


def test_step_from_restore_and_state_checks():
    nx, ny = 64, 24
    rho, ux, uy = inputs.random_state((ny, nx), seed=3, umax=0.05)
    a = lks.Lattice(9, nx, ny, "f32", tau=0.7, layout="planes")
    b = lks.Lattice(9, nx, ny, "f32", tau=0.7, layout="rows")
    a.init(rho, ux, uy)
    # a plane-major state restored into the rows context
    b.restore(a.state.clone())
    _same(a.state, b.state, "restored state")
    sa, sb = a.new_state(), b.new_state()
    assert sb.stride() == b.pop[0].stride() and sa.stride() == a.pop[0].stride()
    a.step_from(a.state, sa)
    b.step_from(b.state, sb)
    torch.cuda.synchronize()
    _same(sa, sb, "step_from")
    # a state in the other layout is refused before anything is launched
    with pytest.raises(ValueError):
        b.step_from(a.state, sb)
    with pytest.raises(ValueError):
        b.step_from(b.state, b.state.contiguous())


def test_adjoint_gradient_layouts_bit_identical():
    rho, ux, uy = inputs.smooth_random(32, seed=3, cutoff=4)
    dev = torch.device("cuda")
    grads = []
    for layout in ("planes", "rows"):
        u = torch.tensor(3 * ux, device=dev, requires_grad=True)
        v = torch.tensor(3 * uy, device=dev, requires_grad=True)
        r = torch.tensor(rho, device=dev)
        L = adjoint.kl_sensor_loss(u, v, r, tau=0.6, nsteps=14, checkpoint=5, dtype="f64",
                                   layout=layout)
        L.backward()
        grads.append((L.detach(), u.grad, v.grad))
    for x, y in zip(*grads):
        _same(x, y, "loss / gradient")


@pytest.mark.parametrize("layout", ["planes", "rows"])
def test_partial_sums_stay_inside_scratch(layout):
    # nx = 300, ny = 2047: the automatic sweep length grows with the tile
    # count, so here the four-cell-wide launch has more workgroups (2047) than
    # the one-cell-wide one (1366); 64 steps of partial sums between two
    # reductions must still fit in lks_scratch_bytes
    nx, ny, steps = 300, 2047, 64
    cfg = lks.make_config(9, nx, ny, "f32", tau=0.6, max_steps=steps, layout=layout)
    nsb = lks.scratch_bytes(cfg)
    guard = 1 << 20
    dev = torch.device("cuda")
    scratch = torch.full((nsb + guard,), 0x5A, dtype=torch.uint8, device=dev)
    ref = lks.Lattice(9, nx, ny, "f32", tau=0.6, max_steps=steps, layout=layout)
    buf = lks.Buffers()
    buf.pop[0], buf.pop[1] = ref.pop[0].data_ptr(), ref.pop[1].data_ptr()
    sensors, flags = torch.zeros_like(ref.sensors), torch.zeros_like(ref.flags)
    sums = torch.zeros_like(ref.sums)
    buf.sensors, buf.flags, buf.sums = sensors.data_ptr(), flags.data_ptr(), sums.data_ptr()
    buf.scratch, buf.scratch_bytes = scratch.data_ptr(), nsb
    L = lks.lib()
    ctx = ctypes.c_void_p()
    assert L.lks_create(ctypes.byref(cfg), ctypes.byref(buf), lks._stream_handle(dev),
                        ctypes.byref(ctx)) == 0
    try:
        rho, ux, uy = inputs.random_state((ny, nx), seed=8, umax=0.05)
        f = [torch.tensor(a, device=dev) for a in (rho, ux, uy)]
        assert L.lks_init_equilibrium(ctx, *[ctypes.c_void_p(t.data_ptr()) for t in f], None) == 0
        assert L.lks_step(ctx, steps, 1) == 0
        torch.cuda.synchronize()
        assert bool((scratch[nsb:] == 0x5A).all()), "partial sums written past lks_scratch_bytes"
        # and the sums are those of an ordinary context on the same state
        ref.init(rho, ux, uy)
        ref.step(steps)
        torch.cuda.synchronize()
        _same(sums, ref.sums, "sums")
    finally:
        L.lks_destroy(ctx)


@pytest.mark.parametrize("dtype,vec,layout", [("f32", 0, "rows"), ("f32", 1, "rows"), ("f64", 0, "rows"),
                                              ("bf16", 0, "rows"), ("f32", 0, "planes")])
def test_d2q9_store_hint_bit_identical(dtype, vec, layout):
    # plain and non-temporal stores of the fused step (the hint the library
    # picks by state size) write the same bytes
    nx, ny, steps = 200, 72, 12
    rho, ux, uy = inputs.random_state((ny, nx), seed=12, umax=0.05)
    thr = np.array([[1e-6, 1e-5], [1e-3, 1e-2], [1e-3, 1e-2], [np.inf, np.inf]])
    out = []
    for nt in (1, 2):
        lat = lks.Lattice(9, nx, ny, dtype, tau=0.6, thr=thr, flag_mask=7, max_steps=steps,
                          launch_vec=vec, layout=layout, launch_nt=nt)
        lat.init(rho, ux, uy)
        lat.step(steps)
        out.append(lat)
    torch.cuda.synchronize()
    a, b = out
    _same(a.state, b.state, "state")
    _same(a.sensors, b.sensors, "sensors")
    _same(a.flags, b.flags, "flags")
    _same(a.sums, b.sums, "sums")


@pytest.mark.parametrize("model,ext", [("bgk", None), ("bgk", ["kn", "qf"]), ("ddf", None),
                                       ("ddf", ["comp", "sigma_h"])])
def test_d2q25_store_hint_bit_identical(model, ext):
    # the D2Q25 kernels take the non-temporal hint on grids of whole tiles
    # (FP32): forced on and off on a small grid, the same bytes
    n, steps = 64, 6
    rho, ux, uy, T, states = inputs.riemann_quadrants(n, seed=4)
    dx = 1.0 / n
    kw = dict(model="ddf", gamma=1.4, prandtl=0.71) if model == "ddf" else {}
    thr = np.array([[1e-7, 1e-6], [1e-4, 1e-3], [1e-3, 1e-2], [1e-3, 1e-2]])
    out = []
    for nt in (1, 2):
        lat = lks.Lattice(25, n, n, "f32", mu=1e-3, dt=inputs.riemann_dt(states, dx, gamma=1.4), dx=dx,
                          bc=(1, 1), thr=thr, flag_mask=15, max_steps=steps, ext=ext, launch_nt=nt, **kw)
        lat.init(rho, ux, uy, T)
        lat.step(steps)
        out.append(lat)
    torch.cuda.synchronize()
    a, b = out
    _same(a.state, b.state, "state")
    _same(a.sensors, b.sensors, "sensors")
    _same(a.flags, b.flags, "flags")
    _same(a.sums, b.sums, "sums")
