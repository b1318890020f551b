// common.hip -- lattice-independent kernels: the fixed-order reduction of
// per-workgroup FP64 partial sums into the per-step sums, and the plain copy
// used as the HBM bandwidth yardstick.
#include "lks_device.h"
#include "lks_internal.h"

namespace lks {

// Many workgroups' partials: a first pass sums each chunk of kBlock
// consecutive workgroups of a step (one per thread, then the fixed wave/LDS
// tree) and writes the chunk's sum over the chunk's first partial, which no
// other workgroup reads; the final pass then adds the chunk sums.  Both
// orders are fixed: the result depends only on the launch shape.
__global__ __launch_bounds__(kBlock) void chunk_sums_kernel(double* __restrict__ partials, int nblocks)
{
    double* p = partials + (long long)blockIdx.y * nblocks * kNsums;
    const long long b = (long long)blockIdx.x * kBlock + threadIdx.x;
    double acc[kNsums];
#pragma unroll
    for (int k = 0; k < kNsums; ++k) acc[k] = b < nblocks ? p[b * kNsums + k] : 0.0;
    __shared__ double out[kNsums];
    block_sums(acc, out);
    __syncthreads();
    if (threadIdx.x < kNsums) p[(long long)blockIdx.x * kBlock * kNsums + threadIdx.x] = out[threadIdx.x];
}

// One workgroup per step over n partials `stride` workgroups apart: thread t
// adds partials t, t + 256, ... in order, then the fixed wave/LDS tree.
__global__ __launch_bounds__(kBlock) void finalize_kernel(const double* __restrict__ partials, int nblocks,
                                                     int n, int stride, double* __restrict__ sums,
                                                     long long row0, int max_rows, double mass_ref,
                                                     double energy_ref)
{
    const int step = blockIdx.x;
    const double* p = partials + (long long)step * nblocks * kNsums;
    double acc[kNsums];
#pragma unroll
    for (int k = 0; k < kNsums; ++k) acc[k] = 0.0;
    for (int b = threadIdx.x; b < n; b += kBlock) {
#pragma unroll
        for (int k = 0; k < kNsums; ++k) acc[k] += p[(long long)b * stride * kNsums + k];
    }
    __shared__ double out[kNsums];
    block_sums(acc, out);
    __syncthreads();
    if (threadIdx.x < kNsums) {
        double v = out[threadIdx.x];
        if (threadIdx.x == 0) v += mass_ref;
        if (threadIdx.x == 3) v += energy_ref;
        const long long row = (row0 + step) % max_rows;
        sums[row * kNsums + threadIdx.x] = v;
    }
}

hipError_t launch_finalize(double* partials, int nblocks, int nsteps, double* sums, long long row0,
                           int max_rows, double mass_ref, double energy_ref, hipStream_t s)
{
    if (nsteps <= 0) return hipSuccess;
    int n = nblocks, stride = 1;
    if (nblocks > kBlock) {
        // a single workgroup per step would walk all the partials alone
        // (77 us per batch of 8 steps on 32,768 workgroups)
        n = (nblocks + kBlock - 1) / kBlock;
        stride = kBlock;
        chunk_sums_kernel<<<dim3((unsigned)n, (unsigned)nsteps), dim3(kBlock), 0, s>>>(partials, nblocks);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    finalize_kernel<<<dim3(nsteps), dim3(kBlock), 0, s>>>(partials, nblocks, n, stride, sums, row0, max_rows,
                                                          mass_ref, energy_ref);
    return hipGetLastError();
}

// One float4 per thread over a grid that covers the buffer once: the fastest
// plain copy form measured on gfx950 (many short waves keep the most requests
// in flight), used as the achievable-bandwidth yardstick.
__global__ __launch_bounds__(kBlock) void copy_kernel(const float4* __restrict__ src, float4* __restrict__ dst,
                                                 long long n)
{
    const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

hipError_t launch_copy_probe(void* dst, const void* src, size_t bytes, hipStream_t s)
{
    const long long n = (long long)(bytes / 16);
    if (n == 0) return hipSuccess;
    const long long blocks = (n + kBlock - 1) / kBlock;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    copy_kernel<<<dim3((unsigned)blocks), dim3(kBlock), 0, s>>>((const float4*)src, (float4*)dst, n);
    return hipGetLastError();
}

} // namespace lks

namespace lks {

__global__ __launch_bounds__(kBlock) void zero_kernel(unsigned long long* __restrict__ p, long long n)
{
    const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// clears n 8-byte words with a kernel (no memset node if the caller captures)
hipError_t launch_zero(void* p, long long nwords, hipStream_t s)
{
    if (nwords <= 0) return hipSuccess;
    zero_kernel<<<dim3((unsigned)((nwords + kBlock - 1) / kBlock)), dim3(kBlock), 0, s>>>(
        (unsigned long long*)p, nwords);
    return hipGetLastError();
}

} // namespace lks
