"""lks_step_noalloc (stepping with the library's own device scratch, for
callers that cannot allocate) against lks_step on the same inputs: every
output bit-identical, over consecutive calls that share the per-device
scratch array, the second smaller than the first."""
import numpy as np
import pytest
import torch

from paper_2603_13618_amd import inputs, lks

pytestmark = pytest.mark.gpu


def _pair(kw, fields):
    """Two lattices of one configuration, both at the equilibrium of fields."""
    a = lks.Lattice(**kw)
    b = lks.Lattice(**kw)
    a.init(*fields)
    b.init(*fields)
    return a, b


def _same(a, b, cur_b):
    torch.cuda.synchronize()
    assert torch.equal(a.state, b.pop[cur_b])
    assert torch.equal(a.sensors, b.sensors)
    assert torch.equal(a.flags, b.flags)
    assert torch.equal(a.sums, b.sums)


def _d2q9(nx, ny, seed, dtype, max_steps, launch_steps=0):
    rho, ux, uy = inputs.random_state((ny, nx), seed, (0.95, 1.05), 0.05)
    thr = np.array([[1e-6, 1e-5], [1e-3, 3e-3], [1e-3, 2e-3], [np.inf, np.inf]])
    kw = dict(lattice=9, nx=nx, ny=ny, dtype=dtype, tau=0.6, thr=thr, flag_mask=7,
              max_steps=max_steps, launch_steps=launch_steps)
    return kw, (rho, ux, uy)


def test_noalloc_matches_step_on_consecutive_calls():
    # a larger grid, then a smaller one: the second call reuses the array the
    # first one filled
    for nx, ny, steps, max_steps, dtype in ((1100, 37, 7, 8, "f32"), (64, 48, 5, 3, "f32"),
                                            (30, 9, 4, 4, "f64"), (12, 5, 3, 2, "bf16")):
        print(f"D2Q9 {dtype} {nx}x{ny}, {steps} steps", flush=True)
        kw, fields = _d2q9(nx, ny, nx + ny, dtype, max_steps)
        a, b = _pair(kw, fields)
        a.step(steps)
        cur = lks.step_noalloc(b.cfg, b.pop, b.sensors, b.flags, b.sums, 0, 0, steps)
        assert cur == a.current()[0]
        _same(a, b, cur)
        # continue from the state and step count reached (sums ring wraps)
        a.step(2)
        cur = lks.step_noalloc(b.cfg, b.pop, b.sensors, b.flags, b.sums, cur, steps, 2)
        _same(a, b, cur)


def test_noalloc_unfused_two_step_and_d2q25():
    kw, fields = _d2q9(260, 7, 3, "f32", 6, launch_steps=2)
    a, b = _pair(kw, fields)
    a.step(5)
    cur = lks.step_noalloc(b.cfg, b.pop, b.sensors, b.flags, b.sums, 0, 0, 5)
    _same(a, b, cur)
    kw, fields = _d2q9(96, 40, 4, "f32", 3)
    a, b = _pair(kw, fields)
    a.step(3, fused=False)
    cur = lks.step_noalloc(b.cfg, b.pop, b.sensors, b.flags, b.sums, 0, 0, 3, fused=False)
    _same(a, b, cur)
    # the double distribution keeps its per-cell hand-over in the array too
    for n, model in ((48, "ddf"), (20, "bgk")):
        rho, ux, uy, T, states = inputs.riemann_quadrants(n, seed=1)
        dx = 1.0 / 64
        kw = dict(lattice=25, nx=n, ny=n, dtype="f32", mu=1e-3, dt=inputs.riemann_dt(states, dx),
                  dx=dx, bc=(1, 1), thr=np.full((4, 2), 1e-3), flag_mask=15, max_steps=4, model=model)
        a, b = _pair(kw, (rho, ux, uy, T))
        a.step(4)
        cur = lks.step_noalloc(b.cfg, b.pop, b.sensors, b.flags, b.sums, 0, 0, 4)
        _same(a, b, cur)


def test_noalloc_rejects_what_does_not_fit():
    # one step's partial sums of a 65536^2 FP32 grid (128 MB) exceed the array
    cfg = lks.make_config(9, 65536, 65536, "f32", tau=0.6, layout=lks.LAYOUT_ROWS)
    t = torch.zeros(64, dtype=torch.float32, device="cuda")
    with pytest.raises(lks.LksError) as e:
        lks.step_noalloc(cfg, (t, t[32:]), t, t.view(torch.uint8), t, 0, 0, 1)
    assert e.value.status == 1 and "scratch" in str(e.value)
