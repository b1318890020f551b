"""Regridding hand-off of the refinement flags (Sec. II.B.2, regridding steps
1-2): buffer layers around tagged cells, tag counts on blocking-factor tiles,
and Berger-Rigoutsos clustering of the tagged tiles into rectangular patches
with a minimum grid efficiency.  Plain numpy / Python.

TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU-baseline timing); the
product library never imports it and shares no code with it.

The paper fixes the buffer width (two cells around each patch) and the grid
efficiency (98 % in two dimensions, Sec. IV) and names the clustering
algorithm of Berger and Rigoutsos without spelling it out.  The steps below
follow that algorithm as published (tight bounding box, accept on efficiency,
else cut at a hole of a signature, else at the strongest inflection of its
Laplacian, else bisect), with the tie-breaking rules fixed here so the result
is unique.
"""
import numpy as np


def tag_buffer(levels, b, bc=(0, 0)):
    """Buffer layer: every cell takes the largest refinement level found in
    the (2b+1) x (2b+1) square around it.  levels: uint8 [ny, nx] (bits 0-1
    of the flag map); bc = (bc_x, bc_y), 0 periodic (wrap), 1 outflow (cells
    beyond the edge repeat the edge cell)."""
    lv = np.asarray(levels, np.uint8) & 3
    ny, nx = lv.shape
    out = np.zeros_like(lv)
    for dy in range(-b, b + 1):
        for dx in range(-b, b + 1):
            ys = np.arange(ny) + dy
            xs = np.arange(nx) + dx
            ys = ys % ny if bc[1] == 0 else np.clip(ys, 0, ny - 1)
            xs = xs % nx if bc[0] == 0 else np.clip(xs, 0, nx - 1)
            out = np.maximum(out, lv[np.ix_(ys, xs)])
    return out


def tag_tiles(levels, level, ts):
    """Number of cells with refinement level >= `level` in each ts x ts tile
    (tiles at the high edges may be partial): int32 [ceil(ny/ts), ceil(nx/ts)]."""
    lv = np.asarray(levels, np.uint8) & 3
    ny, nx = lv.shape
    ty, tx = -(-ny // ts), -(-nx // ts)
    out = np.zeros((ty, tx), np.int32)
    tagged = (lv >= level).astype(np.int64)
    for j in range(ty):
        for i in range(tx):
            out[j, i] = tagged[j * ts:(j + 1) * ts, i * ts:(i + 1) * ts].sum()
    return out


def _tile_cells(ts, n, lo, hi):
    """Cells covered by tiles lo..hi-1 along an axis of n cells."""
    return min(hi * ts, n) - lo * ts


def _find_cut(sx, sy, min_tiles):
    """The cut of a box with column signature sx and row signature sy:
    (axis, k), the box splits into [0, k) and [k, n) along axis 0 (x) or 1 (y);
    None when no admissible cut exists.  Both parts keep >= min_tiles tiles.
      1. a hole: k with sig[k] == 0 (cut just before it); the one nearest
         the middle (smallest |2k + 1 - n|), x before y, then the smaller k;
      2. an inflection: k with lap[k-1] * lap[k] < 0, lap[i] = sig[i+1] -
         2 sig[i] + sig[i-1] (1 <= i <= n-2); the largest |lap[k] - lap[k-1]|,
         then nearest the middle (smallest |2k - n|), x before y, smaller k;
      3. a bisection of the longer axis (x on a tie), k = n // 2."""
    sigs = (np.asarray(sx, np.int64), np.asarray(sy, np.int64))
    best = None
    for axis, sig in enumerate(sigs):
        n = len(sig)
        for k in range(n):
            # a hole at k: cut just before it (the high part's tight bounding
            # box then drops it)
            if sig[k] != 0 or k < min_tiles or n - k < min_tiles:
                continue
            key = (abs(2 * k + 1 - n), axis, k)
            if best is None or key < best[0]:
                best = (key, axis, k)
    if best is not None:
        return best[1], best[2]
    for axis, sig in enumerate(sigs):
        n = len(sig)
        if n < 4:
            continue
        lap = sig[2:] - 2 * sig[1:-1] + sig[:-2]          # lap[i - 1] is at tile i
        for k in range(2, n - 1):
            if k < min_tiles or n - k < min_tiles:
                continue
            a, c = lap[k - 2], lap[k - 1]                   # at tiles k - 1 and k
            if a * c < 0:
                key = (-abs(c - a), abs(2 * k - n), axis, k)
                if best is None or key < best[0]:
                    best = (key, axis, k)
    if best is not None:
        return best[1], best[2]
    nx_, ny_ = len(sigs[0]), len(sigs[1])
    axis = 0 if nx_ >= ny_ else 1
    n = nx_ if axis == 0 else ny_
    if n // 2 >= min_tiles and n - n // 2 >= min_tiles:
        return axis, n // 2
    return None


def cluster(counts, ts, nx, ny, eff, min_tiles=1):
    """Berger-Rigoutsos clustering of the tiles with a non-zero count.
    counts: [ty, tx] tagged cells per ts x ts tile of an nx x ny grid.
    Returns boxes (x0, y0, x1, y1) in cells, half-open, in depth-first order
    (the low part of every cut first).  Every accepted box is the tight
    bounding box of its tagged tiles and has efficiency (tagged cells / box
    cells) >= eff, unless no admissible cut is left."""
    W = np.asarray(counts, np.int64)
    boxes = []

    def recurse(i0, j0, i1, j1):
        sub = W[j0:j1, i0:i1]
        cols = np.nonzero(sub.sum(axis=0))[0]
        if cols.size == 0:
            return
        rows = np.nonzero(sub.sum(axis=1))[0]
        i0, i1 = i0 + cols[0], i0 + cols[-1] + 1
        j0, j1 = j0 + rows[0], j0 + rows[-1] + 1
        sub = W[j0:j1, i0:i1]
        tagged = int(sub.sum())
        area = _tile_cells(ts, nx, i0, i1) * _tile_cells(ts, ny, j0, j1)
        if tagged >= eff * area:
            boxes.append((i0 * ts, j0 * ts, min(i1 * ts, nx), min(j1 * ts, ny)))
            return
        cut = _find_cut(sub.sum(axis=0), sub.sum(axis=1), min_tiles)
        if cut is None:
            boxes.append((i0 * ts, j0 * ts, min(i1 * ts, nx), min(j1 * ts, ny)))
            return
        axis, k = cut
        if axis == 0:
            recurse(i0, j0, i0 + k, j1)
            recurse(i0 + k, j0, i1, j1)
        else:
            recurse(i0, j0, i1, j0 + k)
            recurse(i0, j0 + k, i1, j1)

    ty, tx = W.shape
    recurse(0, 0, tx, ty)
    return boxes
