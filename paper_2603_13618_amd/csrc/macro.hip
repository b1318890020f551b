// macro.hip -- the macroscopic (class-1) sensors from moment fields with
// central finite differences on gfx950: the counterparts the paper compares
// its kinetic class-1 sensors with (Sec. III.A, eqs. sensor-TauNS-mac,
// sensor-C-mac, sensor-S-mac, the rate-of-strain and heat-flux forms; the
// derivatives are central differences, Sec. IV).
//
// One thread per cell, FP64 throughout.  With A_ab = d_a u_b:
//   tau = -mu (A + A^T) - lambda (div u) I,  C = sqrt(D)|div u|,
//   S = |A + A^T - (2/D)(div u) I|,  E = |(A + A^T)/2|,  qH = |u . tau|,
//   qF = |kappa grad T|,  qNSF = |-kappa grad T + u . tau|  (Frobenius / 2-norms).
// d/dx a at j = (a[j+1] - a[j-1]) / (2 dx); ghost cells wrap (periodic) or
// repeat the edge cell (zero gradient).  The fields are read straight from
// global memory: the five-point stencil's rows are served by the L2.
#include <cmath>

#include "lks_device.h"
#include "lks_internal.h"

namespace lks {

namespace {

constexpr int kMTX = 64, kMTY = 4;

__device__ __forceinline__ int nbr(int j, int n, int bc)
{
    if (bc == 0) return j < 0 ? j + n : (j >= n ? j - n : j);
    return j < 0 ? 0 : (j >= n ? n - 1 : j);
}

__global__ __launch_bounds__(kMTX * kMTY) void macro_kernel(MacroArgs a, const double* __restrict__ rho,
                                                            const double* __restrict__ ux,
                                                            const double* __restrict__ uy,
                                                            const double* __restrict__ T,
                                                            double* __restrict__ out)
{
    const int tiles_x = (a.nx + kMTX - 1) / kMTX;
    const int X = (blockIdx.x % tiles_x) * kMTX + threadIdx.x % kMTX;
    const int Y = (blockIdx.x / tiles_x) * kMTY + threadIdx.x / kMTX;
    if (X >= a.nx || Y >= a.ny) return;
    const long long nx = a.nx;
    const long long c = (long long)Y * nx + X;
    const long long xm = (long long)Y * nx + nbr(X - 1, a.nx, a.bc_x);
    const long long xp = (long long)Y * nx + nbr(X + 1, a.nx, a.bc_x);
    const long long ym = (long long)nbr(Y - 1, a.ny, a.bc_y) * nx + X;
    const long long yp = (long long)nbr(Y + 1, a.ny, a.bc_y) * nx + X;
    const double h = a.inv2dx;
    const double dxx = (ux[xp] - ux[xm]) * h, dxy = (uy[xp] - uy[xm]) * h;
    const double dyx = (ux[yp] - ux[ym]) * h, dyy = (uy[yp] - uy[ym]) * h;
    const double div = dxx + dyy;
    const double s = a.per_rho ? rho[c] : 1.0;
    const double m = a.mu * s, l = a.lam * s, k = a.kappa * s;
    const double sxx = 2.0 * dxx, syy = 2.0 * dyy, sxy = dxy + dyx;
    const double txx = -m * sxx - l * div, tyy = -m * syy - l * div, txy = -m * sxy;
    const double u = ux[c], v = uy[c];
    const double qhx = u * txx + v * txy, qhy = u * txy + v * tyy;
    double gx = 0.0, gy = 0.0;
    if (a.which & (kMacroQF | kMacroQNSF)) {
        gx = (T[xp] - T[xm]) * h;
        gy = (T[yp] - T[ym]) * h;
    }
    const double val[kNumMacro] = {
        sqrt(txx * txx + tyy * tyy + 2.0 * txy * txy),
        sqrt(2.0) * fabs(div),
        sqrt((sxx - div) * (sxx - div) + (syy - div) * (syy - div) + 2.0 * sxy * sxy),
        0.5 * sqrt(sxx * sxx + syy * syy + 2.0 * sxy * sxy),
        sqrt(qhx * qhx + qhy * qhy),
        sqrt((k * gx) * (k * gx) + (k * gy) * (k * gy)),
        sqrt((qhx - k * gx) * (qhx - k * gx) + (qhy - k * gy) * (qhy - k * gy)),
    };
#pragma unroll
    for (int q = 0; q < kNumMacro; ++q)
        if (a.plane_of[q] >= 0) out[a.plane_of[q] * a.plane + c] = val[q];
}

} // namespace

hipError_t launch_macro(const MacroArgs& a, const double* rho, const double* ux, const double* uy,
                        const double* T, double* out, hipStream_t s)
{
    const long long tiles = (long long)((a.nx + kMTX - 1) / kMTX) * ((a.ny + kMTY - 1) / kMTY);
    if (tiles <= 0 || tiles > 0x7fffffffLL) return hipErrorInvalidValue;
    macro_kernel<<<dim3((unsigned)tiles), dim3(kMTX * kMTY), 0, s>>>(a, rho, ux, uy, T, out);
    return hipGetLastError();
}

} // namespace lks
