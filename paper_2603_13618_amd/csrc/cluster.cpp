// cluster.cpp -- Berger-Rigoutsos clustering of tagged tiles into
// rectangular patches (the paper's regridding step 2, Sec. II.B.2), host C++.
//
// Input: the number of tagged cells of every ts x ts tile of an nx x ny grid
// (the device's tile counts).  A box is the tight bounding box of the tagged
// tiles inside it; it is accepted when its efficiency (tagged cells / cells)
// reaches eff, otherwise cut:
//   1. at a hole of the column or row signature (a tile column / row with no
//      tag), cutting just before it; the hole nearest the middle of its axis
//      (smallest |2k + 1 - n|), x before y, then the lower index;
//   2. else at an inflection of a signature: between tiles k-1 and k where
//      its discrete Laplacian changes strict sign; the largest jump of the
//      Laplacian, then nearest the middle (smallest |2k - n|), x before y,
//      then the lower index;
//   3. else halfway along the longer axis (x on a tie).
// Every cut leaves at least min_tiles tiles on both sides; a box with no
// admissible cut is accepted as it is.  The low part of a cut is clustered
// first, so the output order is depth-first.
//
// Signatures of a box are read from two prefix-sum tables (row-wise and
// column-wise cumulative tile counts), so each costs O(box side), not
// O(box area).
#include <cstdint>
#include <cstdlib>
#include <vector>

#include "lks.h"

namespace {

struct Grid {
    int tx, ty, ts, nx, ny;
    std::vector<int64_t> rowcum;   // rowcum[j][i]: sum of counts[j][0 .. i-1], width tx+1
    std::vector<int64_t> colcum;   // colcum[i][j]: sum of counts[0 .. j-1][i], width ty+1

    int64_t row_sum(int j, int i0, int i1) const
    {
        const int64_t* r = &rowcum[(size_t)j * (tx + 1)];
        return r[i1] - r[i0];
    }
    int64_t col_sum(int i, int j0, int j1) const
    {
        const int64_t* c = &colcum[(size_t)i * (ty + 1)];
        return c[j1] - c[j0];
    }
    int64_t cells(int lo, int hi, int n) const
    {
        const int64_t end = (int64_t)hi * ts < n ? (int64_t)hi * ts : n;
        return end - (int64_t)lo * ts;
    }
};

struct Cut {
    bool found = false;
    int axis = 0, k = 0;
};

// signature along an axis: x = per tile column of the box, y = per tile row
void signatures(const Grid& g, int i0, int j0, int i1, int j1, std::vector<int64_t>& sx,
                std::vector<int64_t>& sy)
{
    sx.resize(i1 - i0);
    sy.resize(j1 - j0);
    for (int i = i0; i < i1; ++i) sx[i - i0] = g.col_sum(i, j0, j1);
    for (int j = j0; j < j1; ++j) sy[j - j0] = g.row_sum(j, i0, i1);
}

Cut find_cut(const std::vector<int64_t>& sx, const std::vector<int64_t>& sy, int min_tiles)
{
    const std::vector<int64_t>* sig[2] = {&sx, &sy};
    Cut best;
    long long bkey0 = 0, bkey1 = 0, bkey2 = 0;
    // 1. holes
    for (int axis = 0; axis < 2; ++axis) {
        const std::vector<int64_t>& s = *sig[axis];
        const int n = (int)s.size();
        for (int k = 0; k < n; ++k) {
            if (s[k] != 0 || k < min_tiles || n - k < min_tiles) continue;
            const long long key = std::llabs(2LL * k + 1 - n);
            // lexicographic (distance, axis, k); axes and k are visited in order
            if (!best.found || key < bkey0) {
                best.found = true;
                best.axis = axis;
                best.k = k;
                bkey0 = key;
            }
        }
    }
    if (best.found) return best;
    // 2. inflections
    for (int axis = 0; axis < 2; ++axis) {
        const std::vector<int64_t>& s = *sig[axis];
        const int n = (int)s.size();
        if (n < 4) continue;
        for (int k = 2; k <= n - 2; ++k) {
            if (k < min_tiles || n - k < min_tiles) continue;
            const long long lap_a = s[k] - 2 * s[k - 1] + s[k - 2];    // at tile k - 1
            const long long lap_b = s[k + 1] - 2 * s[k] + s[k - 1];    // at tile k
            if (!((lap_a < 0 && lap_b > 0) || (lap_a > 0 && lap_b < 0))) continue;
            const long long jump = std::llabs(lap_b - lap_a);
            const long long mid = std::llabs(2LL * k - n);
            const bool better = !best.found || jump > bkey1 || (jump == bkey1 && mid < bkey2);
            if (better) {
                best.found = true;
                best.axis = axis;
                best.k = k;
                bkey1 = jump;
                bkey2 = mid;
            }
        }
    }
    if (best.found) return best;
    // 3. bisection of the longer axis
    const int nx = (int)sx.size(), ny = (int)sy.size();
    const int axis = nx >= ny ? 0 : 1;
    const int n = axis == 0 ? nx : ny;
    if (n / 2 >= min_tiles && n - n / 2 >= min_tiles) {
        best.found = true;
        best.axis = axis;
        best.k = n / 2;
    }
    return best;
}

struct Work {
    int i0, j0, i1, j1;
};

} // namespace

extern "C" lks_status lks_cluster(const int32_t* counts, int32_t nx, int32_t ny, int32_t ts, double eff,
                                  int32_t min_tiles, lks_box* boxes, int32_t max_boxes, int32_t* nboxes)
{
    if (!counts || !nboxes || nx < 1 || ny < 1 || ts < 1 || min_tiles < 1 || max_boxes < 0 ||
        (max_boxes > 0 && !boxes) || !(eff >= 0.0 && eff <= 1.0))
        return LKS_EINVAL;
    Grid g;
    g.ts = ts;
    g.nx = nx;
    g.ny = ny;
    g.tx = (nx + ts - 1) / ts;
    g.ty = (ny + ts - 1) / ts;
    g.rowcum.assign((size_t)g.ty * (g.tx + 1), 0);
    g.colcum.assign((size_t)g.tx * (g.ty + 1), 0);
    for (int j = 0; j < g.ty; ++j)
        for (int i = 0; i < g.tx; ++i) {
            const int64_t c = counts[(size_t)j * g.tx + i];
            if (c < 0) return LKS_EINVAL;
            g.rowcum[(size_t)j * (g.tx + 1) + i + 1] = g.rowcum[(size_t)j * (g.tx + 1) + i] + c;
            g.colcum[(size_t)i * (g.ty + 1) + j + 1] = g.colcum[(size_t)i * (g.ty + 1) + j] + c;
        }

    int32_t n = 0;
    std::vector<Work> stack;          // depth-first, low part of every cut first
    stack.push_back({0, 0, g.tx, g.ty});
    std::vector<int64_t> sx, sy;
    while (!stack.empty()) {
        Work w = stack.back();
        stack.pop_back();
        // tight bounding box of the tagged tiles
        signatures(g, w.i0, w.j0, w.i1, w.j1, sx, sy);
        int a = 0, b = (int)sx.size() - 1;
        while (a <= b && sx[a] == 0) ++a;
        if (a > b) continue;                        // no tag in this box
        while (sx[b] == 0) --b;
        int c = 0, d = (int)sy.size() - 1;
        while (sy[c] == 0) ++c;
        while (sy[d] == 0) --d;
        const int i0 = w.i0 + a, i1 = w.i0 + b + 1, j0 = w.j0 + c, j1 = w.j0 + d + 1;
        signatures(g, i0, j0, i1, j1, sx, sy);
        int64_t tagged = 0;
        for (int64_t v : sx) tagged += v;
        const int64_t area = g.cells(i0, i1, nx) * g.cells(j0, j1, ny);
        Cut cut;
        if (!((double)tagged >= eff * (double)area)) cut = find_cut(sx, sy, min_tiles);
        if (!cut.found) {
            if (n < max_boxes) {
                lks_box& o = boxes[n];
                o.x0 = i0 * ts;
                o.y0 = j0 * ts;
                o.x1 = (int64_t)i1 * ts < nx ? i1 * ts : nx;
                o.y1 = (int64_t)j1 * ts < ny ? j1 * ts : ny;
            }
            ++n;
            continue;
        }
        // push the high part first so the low part is taken next
        if (cut.axis == 0) {
            stack.push_back({i0 + cut.k, j0, i1, j1});
            stack.push_back({i0, j0, i0 + cut.k, j1});
        } else {
            stack.push_back({i0, j0 + cut.k, i1, j1});
            stack.push_back({i0, j0, i1, j0 + cut.k});
        }
    }
    *nboxes = n;
    return n <= max_boxes ? LKS_OK : LKS_EINVAL;
}
