"""GPU parity of the regridding hand-off (buffer layers, tile counts) against
the oracle, bit for bit, and the whole pipeline flags -> buffer -> tile counts
-> clustering on flag maps the fused step produced."""
import numpy as np
import pytest
import torch

from oracle import regrid
from paper_2603_13618_amd import inputs, lks, workloads

from gpu_util import thresholds

pytestmark = pytest.mark.gpu


def _random_flags(ny, nx, seed):
    rng = np.random.default_rng(seed)
    u = rng.random((ny, nx))
    f = (u < 0.03).astype(np.uint8) + (u < 0.005).astype(np.uint8)
    f[u > 0.999] = 0x82                                    # a few fault cells (level 2)
    return f


# (1024 and 1280 wide: interior tiles take the packed word paths)
@pytest.mark.parametrize("q,nx,ny,bc", [(9, 300, 70, (0, 0)), (9, 5, 3, (0, 0)), (25, 257, 130, (1, 1)),
                                        (25, 129, 17, (0, 1)), (25, 64, 64, (1, 0)),
                                        (9, 1024, 40, (0, 0)), (25, 1280, 37, (1, 1))])
@pytest.mark.parametrize("b", [0, 2, 5, 8])
def test_buffer_and_tiles_match_oracle(q, nx, ny, bc, b):
    kw = dict(tau=0.6) if q == 9 else dict(mu=1e-3, dt=1e-4, dx=1e-2, bc=bc)
    lat = lks.Lattice(q, nx, ny, "f32", **kw)
    flags = _random_flags(ny, nx, seed=b + nx)
    d_flags = torch.from_numpy(flags).cuda()
    lv = lat.tag_buffer(b, flags=d_flags)
    want = regrid.tag_buffer(flags, b, bc if q == 25 else (0, 0))
    assert np.array_equal(lv.cpu().numpy(), want)
    for ts in (1, 8, 13, 64):
        for level in (1, 2):
            c = lat.tag_tiles(lv, level, ts).cpu().numpy()
            assert np.array_equal(c, regrid.tag_tiles(want, level, ts)), (ts, level)


def test_api_limits():
    lat = lks.Lattice(9, 32, 32, "f32", tau=0.6)
    with pytest.raises(lks.LksError):
        lat.tag_buffer(9)
    with pytest.raises(lks.LksError):
        lat.tag_buffer(2, flags=lat.flags, out=lat.flags)
    lv = lat.tag_buffer(2)
    with pytest.raises(lks.LksError):
        lat.tag_tiles(lv, 3, 8)
    with pytest.raises(lks.LksError):
        lat.tag_tiles(lv, 1, 65)


def test_pipeline_on_the_double_shear_layer():
    # the flags of the 128^2 double shear layer after 500 steps, then the
    # paper's regridding parameters: 2 buffer cells, 98 % grid efficiency
    n = 128
    rho, ux, uy = inputs.double_shear_layer(n)
    thr = thresholds("C1")
    lat = lks.Lattice(9, n, n, "f64", tau=0.55, thr=thr, flag_mask=3, max_steps=500)
    lat.init(rho, ux, uy)
    lat.step(500)
    lv = lat.tag_buffer(2)
    flags = lat.flags.cpu().numpy()
    want_lv = regrid.tag_buffer(flags, 2)
    assert np.array_equal(lv.cpu().numpy(), want_lv)
    for level in (1, 2):
        c = lat.tag_tiles(lv, level, 4).cpu().numpy()
        assert np.array_equal(c, regrid.tag_tiles(want_lv, level, 4))
        boxes = lks.cluster(c, n, n, 4, 0.98)
        assert boxes == regrid.cluster(c, 4, n, n, 0.98)
        tagged = int((want_lv >= level).sum())
        covered = sum(int((want_lv[y0:y1, x0:x1] >= level).sum()) for x0, y0, x1, y1 in boxes)
        assert covered == tagged and len(boxes) > 0
        print("level", level, "boxes", len(boxes), "tagged", tagged,
              "cells in boxes", sum((x1 - x0) * (y1 - y0) for x0, y0, x1, y1 in boxes), flush=True)


def test_pipeline_at_full_size():
    # the 4096^2 headline workload's flags after 100 fused steps
    wl = workloads.SMOOTH_4096
    n = wl["nx"]
    rho, ux, uy = inputs.smooth_random(n, seed=wl["seed"], cutoff=wl["cutoff"])
    lat = lks.Lattice(9, n, n, "f32", tau=wl["tau"], thr=wl["thr"], flag_mask=wl["flag_mask"],
                      max_steps=100)
    lat.init(rho, ux, uy)
    lat.step(100)
    lv = lat.tag_buffer(2)
    c = lat.tag_tiles(lv, 1, 8)
    torch.cuda.synchronize()
    flags = lat.flags.cpu().numpy()
    want_lv = regrid.tag_buffer(flags, 2)
    assert np.array_equal(lv.cpu().numpy(), want_lv)
    cw = (want_lv >= 1).reshape(n // 8, 8, n // 8, 8).sum(axis=(1, 3))
    assert np.array_equal(c.cpu().numpy(), cw)
    boxes = lks.cluster(c.cpu().numpy(), n, n, 8, 0.98)
    area = sum((x1 - x0) * (y1 - y0) for x0, y0, x1, y1 in boxes)
    tagged = int(cw.sum())
    print("boxes", len(boxes), "tagged", tagged, "efficiency", tagged / area, flush=True)
    assert sum(int(cw[y0 // 8:y1 // 8, x0 // 8:x1 // 8].sum()) for x0, y0, x1, y1 in boxes) == tagged
