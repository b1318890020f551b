"""Reduced-precision storage forms of the fused D2Q9 step.

BF16 and FP16 storage run the same FP32 arithmetic as FP32 storage and differ
only in how populations are loaded and stored: loads are exact widenings and
stores must be IEEE round-to-nearest-even.  Pinned bit for bit: from one state
representable in the 16-bit form, the 16-bit step's stored populations equal
torch's round-to-nearest-even conversion of the FP32-storage step's result,
and the sensors, flags and FP64 sums of the two runs are identical.
"""
import numpy as np
import pytest
import torch

from paper_2603_13618_amd import inputs, lks

pytestmark = pytest.mark.gpu


def _thresholds(s16, nx, ny):
    """30th / 70th percentiles of each sensor after one FP32 step, so that
    every flag level occurs."""
    pre = lks.Lattice(9, nx, ny, "f32", tau=0.55)
    pre.restore(s16.float())
    pre.step(1)
    q = torch.tensor([0.3, 0.7], dtype=torch.float64, device=pre.sensors.device)
    thr = np.full((4, 2), np.inf)
    for k in range(3):
        thr[k] = torch.quantile(pre.sensors[k].double().flatten(), q).cpu().numpy()
    return thr


def _state16(nx, ny, tdt, seed):
    """Equilibrium of random fields plus a perturbation, rounded to tdt."""
    rho, ux, uy = inputs.random_state((ny, nx), seed=seed, umax=0.08)
    eq = lks.Lattice(9, nx, ny, "f32", tau=0.55)
    eq.init(rho, ux, uy)
    d = eq.state.clone()
    d += torch.from_numpy(inputs.perturbation((9, ny, nx), seed + 1, 2e-4)).to(d)
    return d.to(tdt)


@pytest.mark.parametrize("dtype,tdt", [("bf16", torch.bfloat16), ("f16", torch.float16)])
@pytest.mark.parametrize("nx,ny,vec", [(1024, 40, 0), (1024, 40, 4), (100, 37, 2), (100, 37, 1),
                                       (6, 5, 0)])
def test_store_is_rne_of_the_fp32_result(dtype, tdt, nx, ny, vec):
    # vec: cells per thread (0 = the default, 2 for 16-bit storage).  The FP32
    # run takes the same launch shape: each thread adds its cells' sums before
    # widening them to FP64, so equal sums need equal cells per thread.
    s16 = _state16(nx, ny, tdt, seed=5)
    thr = _thresholds(s16, nx, ny)
    a = lks.Lattice(9, nx, ny, dtype, tau=0.55, thr=thr, flag_mask=7, launch_vec=vec)
    b = lks.Lattice(9, nx, ny, "f32", tau=0.55, thr=thr, flag_mask=7, launch_vec=vec or 2)
    a.restore(s16)
    b.restore(s16.float())
    a.step(1)
    b.step(1)
    torch.cuda.synchronize()
    got = a.state.view(torch.int16)
    want = b.state.to(tdt).view(torch.int16)
    bad = int((got != want).sum())
    print(dtype, nx, ny, "mismatched stores", bad, flush=True)
    assert bad == 0
    assert torch.equal(a.sensors, b.sensors)
    assert torch.equal(a.flags, b.flags)
    levels = torch.bincount(a.flags.flatten().long(), minlength=3)[:3]
    assert int(levels.min()) > 0, levels                       # every level occurs
    assert torch.equal(a.sums[:1], b.sums[:1])


@pytest.mark.parametrize("dtype,tdt", [("bf16", torch.bfloat16), ("f16", torch.float16)])
def test_init_rounds_to_nearest_even(dtype, tdt):
    # the initialiser rounds the FP64 equilibrium deviation to FP32 and then
    # to the 16-bit form, both to nearest even
    nx, ny = 96, 20
    rho, ux, uy = inputs.random_state((ny, nx), seed=9, umax=0.1)
    a = lks.Lattice(9, nx, ny, dtype, tau=0.6)
    b = lks.Lattice(9, nx, ny, "f32", tau=0.6)
    a.init(rho, ux, uy)
    b.init(rho, ux, uy)
    torch.cuda.synchronize()
    assert torch.equal(a.state.view(torch.int16), b.state.to(tdt).view(torch.int16))
