// regrid.hip -- the regridding hand-off of the refinement flags on gfx950
// (Sec. II.B.2, regridding steps 1-2): buffer layers around tagged cells and
// tag counts on blocking-factor tiles, the input of the patch clustering.
//
// Buffer layer: every cell takes the largest refinement level (flag bits
// 0-1) in the (2b+1) x (2b+1) square around it.  The square maximum is
// separable, so a workgroup stages its output tile plus a b-cell halo in LDS,
// takes the row maximum over 2b+1 columns, then the column maximum over 2b+1
// rows.  Ghost cells follow the lattice's boundary conditions (periodic:
// wrap; outflow: repeat the edge cell).
//
// Levels are handled as 2-bit thermometer codes in the bytes of 32-bit words
// (0, 1, 3 for levels 0, 1, 2), so the maximum is a bitwise OR over four
// cells at once and the x window is a set of byte shifts of neighbouring
// words.
//
// Tile counts: the number of cells at level >= L in each ts x ts tile (the
// tiles at the high edges may be partial): on packed words with popcounts
// and a segmented shuffle reduction where the row length and tile size
// allow it, else one wave per tile.
#include "lks_device.h"
#include "lks_internal.h"

namespace lks {

namespace {

constexpr int kTX = 256;               // output cells per workgroup tile, x (64 words)
#ifndef LKS_BUF_TY
#define LKS_BUF_TY 16
#endif
constexpr int kTY = LKS_BUF_TY;        // and y
constexpr int kMaxB = kMaxBuffer;
constexpr int kWX = kTX / 4;           // output words per tile row
constexpr int kPadW = 4;               // halo words on each side: 16 bytes, so interior rows
                                       // load as whole 16-byte pieces (b <= 8 cells needs 2)
constexpr int kSW = kWX + 2 * kPadW;   // staged words per row (18 pieces of 16 bytes)

__device__ __forceinline__ int wrap_or_clamp(int j, int n, int bc)
{
    if (bc == 0) {
        if (j >= -n && j < 2 * n) return j < 0 ? j + n : (j >= n ? j - n : j);   // one period off
        j %= n;                                                                  // tiny grids
        return j < 0 ? j + n : j;
    }
    return j < 0 ? 0 : (j >= n ? n - 1 : j);
}

// Levels 0, 1, 2 as the thermometer codes 0, 1, 3 in each byte: the maximum
// of levels is then the bitwise OR of codes, four cells per 32-bit word.
__device__ __forceinline__ uint32_t to_code(uint32_t flags4)
{
    const uint32_t lv = flags4 & 0x03030303u;
    return lv | ((lv >> 1) & 0x01010101u);
}
__device__ __forceinline__ uint32_t to_level(uint32_t code4)
{
    return (code4 & 0x01010101u) + ((code4 >> 1) & 0x01010101u);
}
// bytes [r, r + 4) of the 8-byte little-endian pair (lo, hi), r in 0..3
__device__ __forceinline__ uint32_t bytes_at(uint32_t lo, uint32_t hi, int r)
{
    return r == 0 ? lo : __builtin_amdgcn_alignbyte(hi, lo, r);
}

// One workgroup: a kTX x kTY output tile.  Stage the tile's codes with a
// b-row and kPadW-word halo in LDS, OR along x over 2b + 1 cells (byte
// shifts of neighbouring words), then along y over 2b + 1 rows.  Each thread
// takes four words (16 cells) at a time through the LDS phases; rows of a
// multiple of 16 cells on 16-byte aligned buffers move 16 bytes per lane in
// and out of HBM.
template <int B>
__global__ __launch_bounds__(kBlock) void buffer_kernel(const uint8_t* __restrict__ flags,
                                                        uint8_t* __restrict__ out, int nx, int ny,
                                                        int bc_x, int bc_y, int tiles_x, int aligned4,
                                                        int aligned16)
{
    constexpr int b = B;
    __shared__ __attribute__((aligned(16))) uint32_t src[kTY + 2 * kMaxB][kSW];
    __shared__ __attribute__((aligned(16))) uint32_t rowor[kTY + 2 * kMaxB][kWX];
    const int X0 = (blockIdx.x % tiles_x) * kTX;
    const int Y0 = (blockIdx.x / tiles_x) * kTY;
    const int H = kTY + 2 * b;
    // Rows of a multiple of 16 cells on 16-byte aligned buffers load whole
    // 16-byte pieces, the ghost pieces too: a piece starts at a multiple of
    // 16, so off the grid it is a whole piece one period away (periodic) or
    // 16 copies of the edge cell (outflow).  Each thread issues all of its
    // loads before it waits for any.  Otherwise interior tiles of rows whose
    // length is a multiple of 4 load whole words, the rest single cells.
    const bool words = aligned4 && X0 >= 4 * kPadW && X0 + kTX + 4 * kPadW <= nx;
    if (aligned16) {
        constexpr int kP = kSW / 4;                                         // pieces per staged row
        constexpr int kItems = ((kTY + 2 * kMaxB) * kP + kBlock - 1) / kBlock;
        uint4 v[kItems];
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            const int e = threadIdx.x + k * kBlock;
            v[k] = make_uint4(0u, 0u, 0u, 0u);
            if (e < H * kP) {
                const int r = e / kP, q = e % kP;
                const uint8_t* row = flags + (long long)wrap_or_clamp(Y0 + r - b, ny, bc_y) * nx;
                const int gx = X0 + 16 * q - 4 * kPadW;
                if (gx >= 0 && gx < nx) {
                    v[k] = *reinterpret_cast<const uint4*>(row + gx);
                } else if (bc_x == 0) {
                    v[k] = *reinterpret_cast<const uint4*>(row + wrap_or_clamp(gx, nx, 0));
                } else {
                    const uint32_t c = (uint32_t)row[gx < 0 ? 0 : nx - 1] * 0x01010101u;
                    v[k] = make_uint4(c, c, c, c);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            const int e = threadIdx.x + k * kBlock;
            if (e < H * kP) {
                const int r = e / kP, q = e % kP;
                *reinterpret_cast<uint4*>(&src[r][4 * q]) =
                    make_uint4(to_code(v[k].x), to_code(v[k].y), to_code(v[k].z), to_code(v[k].w));
            }
        }
    } else {
        for (int e = threadIdx.x; e < H * kSW; e += kBlock) {
            const int r = e / kSW, w = e % kSW;
            const int gy = wrap_or_clamp(Y0 + r - b, ny, bc_y);
            const uint8_t* row = flags + (long long)gy * nx;
            uint32_t v;
            if (words) {
                v = *reinterpret_cast<const uint32_t*>(row + X0 + 4 * (w - kPadW));
            } else {
                v = 0;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int gx = wrap_or_clamp(X0 + 4 * (w - kPadW) + k, nx, bc_x);
                    v |= (uint32_t)row[gx] << (8 * k);
                }
            }
            src[r][w] = to_code(v);
        }
    }
    __syncthreads();
    // words 4c .. 4c + 3 of a row: cell 4w + j of the tile sits in staged word
    // w + kPadW, and its x window (shifts -b .. b, |shift| <= 8 cells) lies in
    // staged words w + kPadW - 2 .. w + kPadW + 2, so the four outputs read
    // staged words 4c + 2 .. 4c + 9, inside the three pieces 4c .. 4c + 11
    for (int e = threadIdx.x; e < H * (kWX / 4); e += kBlock) {
        const int r = e / (kWX / 4), c = e % (kWX / 4);
        const uint4 p0 = *reinterpret_cast<const uint4*>(&src[r][4 * c]);
        const uint4 p1 = *reinterpret_cast<const uint4*>(&src[r][4 * c + 4]);
        const uint4 p2 = *reinterpret_cast<const uint4*>(&src[r][4 * c + 8]);
        const uint32_t win[12] = {p0.x, p0.y, p0.z, p0.w, p1.x, p1.y, p1.z, p1.w, p2.x, p2.y, p2.z, p2.w};
        uint32_t m[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            m[j] = 0;
#pragma unroll
            for (int sh = -b; sh <= b; ++sh) {
                const int p = 4 * (j + kPadW) + sh;    // byte offset of the shifted word in the pieces
                const int q = p >> 2, rr = p & 3;
                m[j] |= bytes_at(win[q], win[q + 1], rr);
            }
        }
        *reinterpret_cast<uint4*>(&rowor[r][4 * c]) = make_uint4(m[0], m[1], m[2], m[3]);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kTY * (kWX / 4); e += kBlock) {
        const int r = e / (kWX / 4), c = e % (kWX / 4);
        const int y = Y0 + r, x = X0 + 16 * c;
        if (y >= ny || x >= nx) continue;
        uint4 m = make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
        for (int k = 0; k <= 2 * b; ++k) {
            const uint4 v = *reinterpret_cast<const uint4*>(&rowor[r + k][4 * c]);
            m.x |= v.x;
            m.y |= v.y;
            m.z |= v.z;
            m.w |= v.w;
        }
        const uint32_t lv[4] = {to_level(m.x), to_level(m.y), to_level(m.z), to_level(m.w)};
        uint8_t* dst = out + (long long)y * nx + x;
        if (aligned16 && x + 16 <= nx) {
            *reinterpret_cast<uint4*>(dst) = make_uint4(lv[0], lv[1], lv[2], lv[3]);
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int xj = x + 4 * j;
                if (xj >= nx) break;
                if (aligned4 && xj + 4 <= nx) {
                    *reinterpret_cast<uint32_t*>(dst + 4 * j) = lv[j];
                } else {
                    for (int k = 0; k < 4 && xj + k < nx; ++k) dst[4 * j + k] = (uint8_t)(lv[j] >> (8 * k));
                }
            }
        }
    }
}

// Tile counts, general form: one wave per tile, lanes stride over its cells.
__global__ __launch_bounds__(kBlock) void tiles_kernel(const uint8_t* __restrict__ levels,
                                                       int* __restrict__ counts, int nx, int ny,
                                                       int level, int ts, int tiles_x, int ntiles)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int tile = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    if (tile >= ntiles) return;                     // whole waves leave together
    const int X0 = (tile % tiles_x) * ts, Y0 = (tile / tiles_x) * ts;
    const int w = min(ts, nx - X0), h = min(ts, ny - Y0);
    int n = 0;
    for (int e = lane; e < w * h; e += kWave) {
        const int r = e / w, c = e % w;
        n += (levels[(long long)(Y0 + r) * nx + X0 + c] & 3) >= level;
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) n += __shfl_xor(n, off, kWave);
    if (lane == 0) counts[tile] = n;
}

// Tile counts on packed words (nx a multiple of 256, ts in 4, 8, .., 64): each
// thread counts one 4-cell word per row of its tile column segment; the
// ts/4 words x ts rows of a tile are spread over a group of lanes and reduced
// with shuffles.  Thread t of the grid owns word column wc and tile row ty.
__global__ __launch_bounds__(kBlock) void tiles_words_kernel(const uint8_t* __restrict__ levels,
                                                             int* __restrict__ counts, int nx, int ny,
                                                             int level, int ts, int tiles_x, int tiles_y)
{
    const int wpt = ts / 4;                         // words per tile row (1 .. 16)
    const int words_x = nx / 4;
    const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    const int wc = (int)(t % words_x);              // word column
    const int ty = (int)(t / words_x);              // tile row
    const bool live = ty < tiles_y;
    int n = 0;
    if (live) {
        const int y0 = ty * ts, y1 = min(y0 + ts, ny);
        const uint32_t* col = reinterpret_cast<const uint32_t*>(levels) + wc;
        for (int y = y0; y < y1; ++y) {
            const uint32_t lv = col[(long long)y * words_x] & 0x03030303u;
            const uint32_t hit = level == 1 ? ((lv | (lv >> 1)) & 0x01010101u) : ((lv >> 1) & 0x01010101u);
            n += __builtin_popcount(hit);
        }
    }
    // lanes wc .. wc + wpt - 1 of one tile are adjacent (words_x is a
    // multiple of wpt unless the last tile is partial, handled by the mask)
    const int lane = threadIdx.x & (kWave - 1);
    for (int off = 1; off < wpt; off <<= 1) {
        const int other = __shfl_down(n, off, kWave);
        n += (lane % wpt) + off < wpt ? other : 0;
    }
    if (live && wc % wpt == 0) counts[(long long)ty * tiles_x + wc / wpt] = n;
}

} // namespace

hipError_t launch_tag_buffer(const uint8_t* flags, uint8_t* out, int nx, int ny, int bc_x, int bc_y,
                             int b, hipStream_t s)
{
    if (b < 0 || b > kMaxB) return hipErrorInvalidValue;
    const int tiles_x = (nx + kTX - 1) / kTX, tiles_y = (ny + kTY - 1) / kTY;
    // whole words need rows of a multiple of 4 bytes on 4-byte aligned
    // buffers, whole 16-byte pieces rows of a multiple of 16 on 16-byte
    // aligned ones
    const int aligned4 = ((uintptr_t)flags % 4 == 0) && ((uintptr_t)out % 4 == 0) && nx % 4 == 0;
    const int aligned16 = ((uintptr_t)flags % 16 == 0) && ((uintptr_t)out % 16 == 0) && nx % 16 == 0;
    const dim3 grid((unsigned)(tiles_x * tiles_y)), block(kBlock);
    switch (b) {
#define LKS_BUFFER_CASE(B)                                                                          \
    case B:                                                                                         \
        buffer_kernel<B><<<grid, block, 0, s>>>(flags, out, nx, ny, bc_x, bc_y, tiles_x, aligned4, aligned16); \
        break;
        LKS_BUFFER_CASE(0) LKS_BUFFER_CASE(1) LKS_BUFFER_CASE(2) LKS_BUFFER_CASE(3) LKS_BUFFER_CASE(4)
        LKS_BUFFER_CASE(5) LKS_BUFFER_CASE(6) LKS_BUFFER_CASE(7) LKS_BUFFER_CASE(8)
#undef LKS_BUFFER_CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_tag_tiles(const uint8_t* levels, int* counts, int nx, int ny, int level, int ts,
                            hipStream_t s)
{
    const int tiles_x = (nx + ts - 1) / ts, tiles_y = (ny + ts - 1) / ts;
    // packed path: whole words, tiles of 4 .. 64 cells aligned to the wave's
    // lane groups (64 / (ts/4) tiles per wave)
    const int wpt = ts / 4;
    if ((uintptr_t)levels % 4 == 0 && nx % 4 == 0 && ts % 4 == 0 && (wpt & (wpt - 1)) == 0 &&
        (nx / 4) % kWave == 0) {
        const long long threads = (long long)(nx / 4) * tiles_y;
        tiles_words_kernel<<<dim3((unsigned)((threads + kBlock - 1) / kBlock)), dim3(kBlock), 0, s>>>(
            levels, counts, nx, ny, level, ts, tiles_x, tiles_y);
        return hipGetLastError();
    }
    const int ntiles = tiles_x * tiles_y;
    const int per_block = kBlock / kWave;
    tiles_kernel<<<dim3((unsigned)((ntiles + per_block - 1) / per_block)), dim3(kBlock), 0, s>>>(
        levels, counts, nx, ny, level, ts, tiles_x, ntiles);
    return hipGetLastError();
}

} // namespace lks
