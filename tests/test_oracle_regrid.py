"""Pins of the regridding oracle (buffer layers, tile counts, Berger-Rigoutsos
clustering) against library routines, exact constructions and the invariants
a valid patch set must satisfy."""
import numpy as np
import pytest
import scipy.ndimage as ndi

from oracle import regrid


def _levels(shape, seed, p1=0.05, p2=0.01):
    rng = np.random.default_rng(seed)
    u = rng.random(shape)
    return (u < p1).astype(np.uint8) + (u < p2).astype(np.uint8)


@pytest.mark.parametrize("bc", [(0, 0), (1, 1), (0, 1), (1, 0)])
@pytest.mark.parametrize("b", [0, 1, 2, 3])
def test_buffer_is_a_maximum_filter(bc, b):
    lv = _levels((23, 31), seed=b)
    lv[3, 5] |= 0x80                                   # the fault bit is not a level
    got = regrid.tag_buffer(lv, b, bc)
    # the same filter from scipy, axis by axis (rows: bc_y, columns: bc_x)
    mode = ["wrap" if bc[1] == 0 else "nearest", "wrap" if bc[0] == 0 else "nearest"]
    want = ndi.maximum_filter(lv & 3, size=2 * b + 1, mode=mode)
    assert np.array_equal(got, want)


def test_buffer_of_one_cell_is_a_square():
    lv = np.zeros((20, 20), np.uint8)
    lv[10, 4] = 2
    got = regrid.tag_buffer(lv, 2)
    assert got.sum() == 2 * 25 and (got[8:13, 2:7] == 2).all()
    got = regrid.tag_buffer(lv, 2, bc=(0, 0))
    lv[0, 0] = 1
    got = regrid.tag_buffer(lv, 1, bc=(0, 0))              # wraps to the far corner
    assert got[19, 19] == 1 and got[1, 1] == 1 and got[2, 2] == 0


@pytest.mark.parametrize("ts", [1, 4, 8, 16])
def test_tile_counts(ts):
    lv = _levels((37, 50), seed=ts)
    for level in (1, 2):
        c = regrid.tag_tiles(lv, level, ts)
        assert c.sum() == (lv >= level).sum()
        # against a padded reshape-sum
        ty, tx = c.shape
        pad = np.zeros((ty * ts, tx * ts), np.int64)
        pad[:37, :50] = lv >= level
        assert np.array_equal(c, pad.reshape(ty, ts, tx, ts).sum(axis=(1, 3)))


def _check_patches(counts, ts, nx, ny, boxes, eff):
    """Invariants of a patch set: disjoint, covering every tagged tile, tight
    (each edge row / column holds a tag) and efficient unless uncuttable."""
    W = np.asarray(counts)
    cover = np.zeros(W.shape, int)
    for (x0, y0, x1, y1) in boxes:
        assert x0 % ts == 0 and y0 % ts == 0 and 0 <= x0 < x1 <= nx and 0 <= y0 < y1 <= ny
        i0, j0, i1, j1 = x0 // ts, y0 // ts, -(-x1 // ts), -(-y1 // ts)
        cover[j0:j1, i0:i1] += 1
        sub = W[j0:j1, i0:i1]
        assert sub[:, 0].sum() and sub[:, -1].sum() and sub[0, :].sum() and sub[-1, :].sum()
        # with cuts down to one tile, only a single tile can stay below eff
        e = sub.sum() / ((x1 - x0) * (y1 - y0))
        assert e >= eff or (i1 - i0 == 1 and j1 - j0 == 1)
    assert cover.max() <= 1                                   # disjoint
    assert (cover[W > 0] == 1).all()                          # every tag covered


def test_one_rectangle_is_one_box():
    W = np.zeros((10, 12), np.int32)
    W[2:5, 3:9] = 16
    boxes = regrid.cluster(W, 4, 48, 40, 0.98)
    assert boxes == [(12, 8, 36, 20)]


def test_separate_rectangles_split_at_the_hole():
    W = np.zeros((10, 12), np.int32)
    W[1:4, 1:4] = 16
    W[6:9, 7:11] = 16
    boxes = regrid.cluster(W, 4, 48, 40, 0.98)
    assert sorted(boxes) == [(4, 4, 16, 16), (28, 24, 44, 36)]


def test_l_shape_splits_at_the_inflection():
    # an L of full tiles: two boxes of efficiency 1 that cover it exactly
    W = np.zeros((12, 12), np.int32)
    W[1:3, 1:11] = 64
    W[3:11, 1:3] = 64
    boxes = regrid.cluster(W, 8, 96, 96, 0.98)
    assert len(boxes) == 2
    area = sum((x1 - x0) * (y1 - y0) for x0, y0, x1, y1 in boxes)
    assert area == (W > 0).sum() * 64
    _check_patches(W, 8, 96, 96, boxes, 0.98)


@pytest.mark.parametrize("seed", range(6))
def test_random_blobs_give_valid_patches(seed):
    rng = np.random.default_rng(seed)
    lv = np.zeros((96, 80), np.uint8)
    for _ in range(5):
        cy, cx, r = rng.integers(0, 96), rng.integers(0, 80), rng.integers(3, 12)
        yy, xx = np.ogrid[:96, :80]
        lv[(yy - cy) ** 2 + (xx - cx) ** 2 <= r * r] = 1
    lv = regrid.tag_buffer(lv, 2, bc=(1, 1))
    for ts, eff in ((4, 0.98), (8, 0.7), (1, 0.98)):
        W = regrid.tag_tiles(lv, 1, ts)
        boxes = regrid.cluster(W, ts, 80, 96, eff)
        _check_patches(W, ts, 80, 96, boxes, eff)
        if ts == 1:
            # with single-cell tiles every box can be cut down to full efficiency
            for (x0, y0, x1, y1) in boxes:
                assert W[y0:y1, x0:x1].sum() >= eff * (x1 - x0) * (y1 - y0)


def test_partial_edge_tiles_count_their_real_cells():
    # a 10 x 10 grid with 8-cell tiles: the edge tiles hold 2 columns / rows
    lv = np.zeros((10, 10), np.uint8)
    lv[8:, 8:] = 1
    W = regrid.tag_tiles(lv, 1, 8)
    assert W.tolist() == [[0, 0], [0, 4]]
    assert regrid.cluster(W, 8, 10, 10, 0.98) == [(8, 8, 10, 10)]


def test_empty_map_has_no_patches():
    assert regrid.cluster(np.zeros((4, 4), np.int32), 8, 32, 32, 0.98) == []
