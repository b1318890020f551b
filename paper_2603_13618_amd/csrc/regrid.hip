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
// Tile counts: the number of cells at level >= L in each ts x ts tile (the
// tiles at the high edges may be partial); one wave per tile, each lane sums
// a strided share of the tile and the wave reduces with shuffles.
#include "lks_device.h"
#include "lks_internal.h"

namespace lks {

namespace {

constexpr int kTX = 128;               // output cells per workgroup tile, x
constexpr int kTY = 16;                // and y
constexpr int kMaxB = kMaxBuffer;

__device__ __forceinline__ int wrap_or_clamp(int j, int n, int bc)
{
    if (bc == 0) {
        j %= n;
        return j < 0 ? j + n : j;
    }
    return j < 0 ? 0 : (j >= n ? n - 1 : j);
}

__global__ __launch_bounds__(kBlock) void buffer_kernel(const uint8_t* __restrict__ flags,
                                                        uint8_t* __restrict__ out, int nx, int ny,
                                                        int bc_x, int bc_y, int b, int tiles_x)
{
    __shared__ uint8_t src[kTY + 2 * kMaxB][kTX + 2 * kMaxB];
    __shared__ uint8_t rowmax[kTY + 2 * kMaxB][kTX];
    const int X0 = (blockIdx.x % tiles_x) * kTX;
    const int Y0 = (blockIdx.x / tiles_x) * kTY;
    const int W = kTX + 2 * b, H = kTY + 2 * b;

    // stage the tile and its halo (levels only)
    for (int e = threadIdx.x; e < W * H; e += kBlock) {
        const int r = e / W, c = e % W;
        const int gy = wrap_or_clamp(Y0 + r - b, ny, bc_y);
        const int gx = wrap_or_clamp(X0 + c - b, nx, bc_x);
        src[r][c] = flags[(long long)gy * nx + gx] & 3;
    }
    __syncthreads();
    // maximum along x over 2b + 1 columns
    for (int e = threadIdx.x; e < kTX * H; e += kBlock) {
        const int r = e / kTX, c = e % kTX;
        uint8_t m = 0;
        for (int k = 0; k <= 2 * b; ++k) m = max(m, src[r][c + k]);
        rowmax[r][c] = m;
    }
    __syncthreads();
    // then along y over 2b + 1 rows
    for (int e = threadIdx.x; e < kTX * kTY; e += kBlock) {
        const int r = e / kTX, c = e % kTX;
        const int x = X0 + c, y = Y0 + r;
        if (x >= nx || y >= ny) continue;
        uint8_t m = 0;
        for (int k = 0; k <= 2 * b; ++k) m = max(m, rowmax[r + k][c]);
        out[(long long)y * nx + x] = m;
    }
}

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

} // namespace

hipError_t launch_tag_buffer(const uint8_t* flags, uint8_t* out, int nx, int ny, int bc_x, int bc_y,
                             int b, hipStream_t s)
{
    if (b < 0 || b > kMaxB) return hipErrorInvalidValue;
    const int tiles_x = (nx + kTX - 1) / kTX, tiles_y = (ny + kTY - 1) / kTY;
    buffer_kernel<<<dim3((unsigned)(tiles_x * tiles_y)), dim3(kBlock), 0, s>>>(flags, out, nx, ny, bc_x,
                                                                              bc_y, b, tiles_x);
    return hipGetLastError();
}

hipError_t launch_tag_tiles(const uint8_t* levels, int* counts, int nx, int ny, int level, int ts,
                            hipStream_t s)
{
    const int tiles_x = (nx + ts - 1) / ts, tiles_y = (ny + ts - 1) / ts;
    const int ntiles = tiles_x * tiles_y;
    const int per_block = kBlock / kWave;
    tiles_kernel<<<dim3((unsigned)((ntiles + per_block - 1) / per_block)), dim3(kBlock), 0, s>>>(
        levels, counts, nx, ny, level, ts, tiles_x, ntiles);
    return hipGetLastError();
}

} // namespace lks
