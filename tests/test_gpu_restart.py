"""Checkpoint and restart: 100 steps in one context equal 50 steps, a copy of
the state to host memory, a new context restored from it, and 50 more steps,
bit for bit (state, sensors, flags and the per-step sums of steps 51-100)."""
import numpy as np
import pytest
import torch

from paper_2603_13618_amd import inputs, lks

pytestmark = pytest.mark.gpu


def _restart(kw, fields, total=100, split=50):
    a = lks.Lattice(max_steps=total, **kw)
    a.init(*fields)
    a.step(total)
    b = lks.Lattice(max_steps=total, **kw)
    b.init(*fields)
    b.step(split)
    host = b.read_host(0)                      # synchronous copy out, [Q, ny, nx]
    del b
    c = lks.Lattice(max_steps=total, **kw)
    c.restore(torch.from_numpy(np.ascontiguousarray(host)).view(c.pop[0].dtype)
              if kw.get("dtype") == "bf16" else torch.from_numpy(np.ascontiguousarray(host)), split)
    c.step(total - split)
    torch.cuda.synchronize()
    assert c.current()[1] == total
    assert torch.equal(a.state, c.state)
    assert torch.equal(a.sensors, c.sensors)
    assert torch.equal(a.flags, c.flags)
    assert torch.equal(a.sums[split:], c.sums[split:])
    assert a.check() == c.check()


@pytest.mark.parametrize("dtype", ["f32", "bf16", "f64"])
def test_d2q9_restart_is_bit_identical(dtype):
    rho, ux, uy = inputs.smooth_random(192, seed=3, cutoff=8)
    thr = np.array([[1e-7, 1e-6], [1e-4, 3e-4], [1e-4, 3e-4], [np.inf, np.inf]])
    _restart(dict(lattice=9, nx=192, ny=160, dtype=dtype, tau=0.52, thr=thr, flag_mask=7),
             (rho[:160], ux[:160], uy[:160]))


def test_d2q25_restart_is_bit_identical():
    n = 96
    rho, ux, uy, T, states = inputs.riemann_quadrants(n, seed=0)
    dx = 1.0 / n
    thr = np.array([[1e-7, 1e-6], [1e-4, 1e-3], [1e-3, 1e-2], [1e-3, 1e-2]])
    for model in ("bgk", "ddf"):
        _restart(dict(lattice=25, nx=n, ny=n, dtype="f32", mu=1e-3, dt=inputs.riemann_dt(states, dx),
                      dx=dx, bc=(1, 1), thr=thr, flag_mask=15, model=model), (rho, ux, uy, T))
