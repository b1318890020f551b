"""The library's host clustering (lks_cluster, C++) against the oracle's
Berger-Rigoutsos reading: identical patch lists, box for box.  Runs on the
CPU (no GPU needed)."""
import numpy as np
import pytest

from oracle import regrid
from paper_2603_13618_amd import lks


def _blobs(ny, nx, seed, n=6):
    rng = np.random.default_rng(seed)
    lv = np.zeros((ny, nx), np.uint8)
    yy, xx = np.ogrid[:ny, :nx]
    for _ in range(n):
        cy, cx, r = rng.integers(0, ny), rng.integers(0, nx), rng.integers(2, 14)
        lv[(yy - cy) ** 2 + (xx - cx) ** 2 <= r * r] = rng.integers(1, 3)
    return lv


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("ts,eff,min_tiles", [(1, 0.98, 1), (4, 0.98, 1), (8, 0.7, 1), (4, 0.9, 2),
                                              (16, 0.98, 1)])
def test_library_clustering_equals_oracle(seed, ts, eff, min_tiles):
    ny, nx = 100, 131
    lv = regrid.tag_buffer(_blobs(ny, nx, seed), 2, bc=(1, 0))
    for level in (1, 2):
        W = regrid.tag_tiles(lv, level, ts)
        want = regrid.cluster(W, ts, nx, ny, eff, min_tiles)
        got = lks.cluster(W, nx, ny, ts, eff, min_tiles)
        assert got == want


def test_edge_cases_and_errors():
    assert lks.cluster(np.zeros((3, 3), np.int32), 20, 20, 8) == []
    W = np.zeros((4, 5), np.int32)
    W[3, 4] = 1
    assert lks.cluster(W, 37, 29, 8, 0.98) == regrid.cluster(W, 8, 37, 29, 0.98) == [(32, 24, 37, 29)]
    W = (np.arange(64).reshape(8, 8) % 3 == 0).astype(np.int32)      # scattered single tiles
    with pytest.raises(lks.LksError):
        lks.cluster(W, 8, 8, 1, 0.98, max_boxes=2)
    assert lks.cluster(W, 8, 8, 1, 0.98) == regrid.cluster(W, 1, 8, 8, 0.98)
    with pytest.raises(lks.LksError):
        lks.cluster(W, 8, 8, 1, 1.5)
