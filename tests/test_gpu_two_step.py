"""Two fused D2Q9 steps per launch (launch_steps = 2, temporal blocking)
against one step per launch: the same per-cell arithmetic, so the state,
the last step's sensors and flags and the positivity-fault count must be
bit-identical.  The per-step FP64 sums group the cells differently: the
one-step kernels add each group of up to four cells in the arithmetic type
before widening, the two-step kernel widens every cell, so with FP32
arithmetic the two differ by at most about 3 * 2^-24 * sum |term| (2^-21 is
used), with FP64 arithmetic by FP64 rounding only.  Odd step counts end on a
one-step launch of the same strips."""
import numpy as np
import pytest
import torch

from paper_2603_13618_amd import inputs, lks

pytestmark = pytest.mark.gpu


def _same(a, b, what):
    a, b = a.detach().cpu(), b.detach().cpu()
    if a.dtype in (torch.bfloat16, torch.float16):
        a, b = a.view(torch.int16), b.view(torch.int16)
    assert torch.equal(a, b) or bool(((a == b) | (a.isnan() & b.isnan())).all()), what


def _run(dtype, nx, ny, steps, layout, launch_steps, fields, thr, mask, state=None):
    lat = lks.Lattice(9, nx, ny, dtype, tau=0.6, thr=thr, flag_mask=mask, max_steps=max(steps, 1),
                      layout=layout, launch_steps=launch_steps)
    if state is None:
        lat.init(*fields)
    else:
        lat.restore(state)
    lat.step(steps)
    torch.cuda.synchronize()
    return lat


@pytest.mark.parametrize("dtype", ["f32", "f64", "bf16", "f16"])
@pytest.mark.parametrize("nx,ny,layout", [(200, 72, "rows"), (130, 17, "planes"), (64, 64, "rows"),
                                          (3, 5, "rows"), (1, 1, "planes")])
@pytest.mark.parametrize("steps", [1, 2, 7])
def test_two_step_launches_bit_identical(dtype, nx, ny, layout, steps):
    fields = inputs.random_state((ny, nx), seed=nx + steps, umax=0.05)
    thr = np.array([[1e-6, 1e-5], [1e-3, 1e-2], [1e-3, 1e-2], [np.inf, np.inf]])
    mask = lks.S_KL | lks.S_NEQ | lks.S_PI
    a = _run(dtype, nx, ny, steps, layout, 0, fields, thr, mask)
    b = _run(dtype, nx, ny, steps, layout, 2, fields, thr, mask)
    _same(a.state, b.state, "state")
    _same(a.sensors, b.sensors, "sensors")
    _same(a.flags, b.flags, "flags")
    sa, sb = a.sums.cpu().numpy(), b.sums.cpu().numpy()
    # sum |term| per column: mass and the sensors are nonnegative; a momentum
    # term is below rho |u| <= 0.2 per cell for these fields
    scale = np.abs(sa)
    scale[:, 1:3] += 0.2 * nx * ny
    rel = 1e-14 if dtype == "f64" else 2.0 ** -21
    assert np.all(np.abs(sa - sb) <= rel * scale + 1e-300), np.abs(sa - sb).max()
    assert a.check() == b.check() == 0
    # the state changes buffer once per launch: steps // 2 pairs, then an odd step alone
    assert a.current() == (steps % 2, steps)
    assert b.current() == ((steps // 2 + steps % 2) % 2, steps)


def test_two_step_counts_faults_of_both_steps(orc):
    n = 24
    rho, ux, uy = inputs.random_state((n, n), 3, (0.99, 1.01), 0.01)
    f = orc.equilibrium(9, rho, ux, uy)
    _, _, w = orc.lattice(9)
    f[2, 5, 7] = -0.01                          # a negative population, moved by the stream
    d = torch.from_numpy(f - w[:, None, None]).float()
    counts = []
    for ls in (0, 2):
        lat = lks.Lattice(9, n, n, "f32", tau=0.6, max_steps=4, launch_steps=ls)
        lat.restore(d)
        lat.step(4)
        torch.cuda.synchronize()
        counts.append(lat.check())
        if ls == 0:
            ref = lat
        else:
            _same(ref.state, lat.state, "state")
            _same(ref.flags, lat.flags, "flags")
    assert counts[0] == counts[1] > 0


def test_two_step_bit_identical_past_2_31_elements():
    """16384^2 FP32 (9 x 2^28 population elements per state): two steps per
    launch against one, compared on the device."""
    n = 16384
    rho, ux, uy = inputs.smooth_random(n, seed=1, cutoff=8)
    thr = np.array([[1e-6, 1e-5], [1e-3, 1e-2], [1e-3, 1e-2], [np.inf, np.inf]])
    mask = lks.S_KL | lks.S_NEQ | lks.S_PI
    lats = []
    for ls in (0, 2):
        lat = lks.Lattice(9, n, n, "f32", tau=0.52, thr=thr, flag_mask=mask, max_steps=2, launch_steps=ls)
        lat.init(rho, ux, uy)
        lat.step(2)
        torch.cuda.synchronize()
        lats.append(lat)
    a, b = lats
    assert torch.equal(a.state, b.state)
    assert torch.equal(a.sensors, b.sensors)
    assert torch.equal(a.flags, b.flags)
    assert a.check() == b.check() == 0
    sa, sb = a.sums.cpu().numpy(), b.sums.cpu().numpy()
    scale = np.abs(sa)
    scale[:, 1:3] += 0.2 * n * n
    assert np.all(np.abs(sa - sb) <= 2.0 ** -21 * scale + 1e-300)
