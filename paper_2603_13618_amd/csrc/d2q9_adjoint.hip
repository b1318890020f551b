// d2q9_adjoint.hip -- hand-written reverse mode of the D2Q9 step for the
// gradient of the summed smooth KL sensor with respect to the initial
// velocity field.
//
// Forward (per step n): g_n(x)_i = f_{n-1}(x - c_i)_i (pull streaming),
// f_n = C(g_n) = g_n - (g_n - f^eq(g_n))/tau, with f^eq_i = w_i rho P_i(u),
// P_i = 1 + 3 c_i.u + 9/2 (c_i.u)^2 - 3/2 u^2 (order-2 Grad-Hermite
// equilibrium, Sec. II.A.3).  Loss L = sum_x S_KL(g_N(x)), S_KL =
// sum_i [g_i ln(g_i/f^eq_i) - g_i + f^eq_i] (eq. HKL-sensor).
//
// Reverse, with dP_i/du_a = 3 c_ia + 9 (c_i.u) c_ia - 3 u_a:
//   seed   dL/dg_N,j = ln(g_j/f^eq_j) - sum_a B'_a (c_ja - u_a)/rho,
//          B'_a = sum_i (g_i/f^eq_i) w_i rho dP_i/du_a
//          (the derivative through rho vanishes because sum f^eq = sum g);
//   stream dL/df_n,i(x) = dL/dg_{n+1},i(x + c_i)  (a pull by +c_i);
//   collide dL/dg_n,j = (1 - 1/tau) l_j + (1/tau) [sum_i l_i w_i P_i
//          + sum_a B_a (c_ja - u_a)/rho],  B_a = sum_i l_i w_i rho dP_i/du_a,
//          with l = dL/df_n;
//   init   dL/du0_a = sum_i l_i w_i rho0 dP_i/du_a(u0), l = dL/df_0.
// Each reverse step reads the previous state (pulled by -c), the incoming
// adjoint (pulled by +c) and writes the outgoing adjoint: no atomics, every
// output written once.
#include "lks_device.h"
#include "lks_internal.h"

namespace lks {

__device__ __forceinline__ constexpr int acx(int i) { return i / 3 - 1; }
__device__ __forceinline__ constexpr int acy(int i) { return i % 3 - 1; }
template <typename R>
__device__ __forceinline__ constexpr R aw(int i)
{
    return (i == 4) ? R(4.0 / 9.0) : ((acx(i) == 0 || acy(i) == 0) ? R(1.0 / 9.0) : R(1.0 / 36.0));
}

template <int N, typename F, int I = 0>
__device__ __forceinline__ void sfor(F&& f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        sfor<N, F, I + 1>(static_cast<F&&>(f));
    }
}

// one cell's x-shifted read: out = row[(x - CX) mod nx], scalar loads
template <int CX, typename R>
__device__ __forceinline__ R shifted(const R* __restrict__ row, int x, int nx)
{
    int xs = x - CX;
    xs = xs < 0 ? xs + nx : (xs >= nx ? xs - nx : xs);
    return row[xs];
}

template <int SIGN, typename R>
__device__ __forceinline__ void pull9(const R* __restrict__ f, const PopLayout& L, int x, int y, int nx,
                                      int ny, R (&out)[9])
{
    sfor<9>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        constexpr int cx = SIGN * acx(i), cy = SIGN * acy(i);
        int ys = y - cy;
        ys = ys < 0 ? ys + ny : (ys >= ny ? ys - ny : ys);
        out[i] = shifted<cx>(f + L.at(i, ys, 0), x, nx);
    });
}

// moments of a cell from its stored deviations d_i = f_i - w_i rho0
template <typename R>
__device__ __forceinline__ void cell_moments(const R (&d)[9], R rho0, R& drho, R& rho, R& ux, R& uy)
{
    R jx = R(0), jy = R(0);
    drho = R(0);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        drho += d[i];
        jx += R(acx(i)) * d[i];
        jy += R(acy(i)) * d[i];
    }
    rho = rho0 + drho;
    ux = jx / rho;
    uy = jy / rho;
}

template <typename R>
__global__ __launch_bounds__(kBlock) void adj_seed_kernel(int nx, int ny, long long plane, PopLayout L, R rho0,
                                                     const R* __restrict__ fprev,
                                                     R* __restrict__ lam)
{
    const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (c >= plane) return;
    const int x = (int)(c % nx), y = (int)(c / nx);
    R d[9], drho, rho, ux, uy;
    pull9<1>(fprev, L, x, y, nx, ny, d);
    cell_moments(d, rho0, drho, rho, ux, uy);
    const R usq15 = R(1.5) * (ux * ux + uy * uy);
    // with x_i = f^neq_i / f^eq_i: g_i / f^eq_i = 1 + x_i, and the "1" part of
    // B'_a vanishes because sum_i w_i dP_i/du_a = 0
    R bx = R(0), by = R(0), lnr[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const R cu = R(acx(i)) * ux + R(acy(i)) * uy;
        const R deq = aw<R>(i) * (drho + rho * (cu * (R(3) + R(4.5) * cu) - usq15));
        const R feq = aw<R>(i) * rho0 + deq;
        const R xi = (d[i] - deq) / feq;
        lnr[i] = kl_dphi(xi);
        const R k = R(3) + R(9) * cu;
        bx += xi * aw<R>(i) * rho * (k * R(acx(i)) - R(3) * ux);
        by += xi * aw<R>(i) * rho * (k * R(acy(i)) - R(3) * uy);
    }
#pragma unroll
    for (int j = 0; j < 9; ++j)
        lam[L.at(j, y, x)] = lnr[j] - (bx * (R(acx(j)) - ux) + by * (R(acy(j)) - uy)) / rho;
}

template <typename R>
__global__ __launch_bounds__(kBlock) void adj_step_kernel(int nx, int ny, long long plane, PopLayout L, R rho0, R tau,
                                                     const R* __restrict__ fprev,
                                                     const R* __restrict__ lam_in,
                                                     R* __restrict__ lam_out)
{
    const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (c >= plane) return;
    const int x = (int)(c % nx), y = (int)(c / nx);
    R d[9], l[9], drho, rho, ux, uy;
    pull9<1>(fprev, L, x, y, nx, ny, d);
    pull9<-1>(lam_in, L, x, y, nx, ny, l);
    cell_moments(d, rho0, drho, rho, ux, uy);
    const R usq = ux * ux + uy * uy;
    R a0 = R(0), bx = R(0), by = R(0);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const R cu = R(acx(i)) * ux + R(acy(i)) * uy;
        const R P = R(1) + cu * (R(3) + R(4.5) * cu) - R(1.5) * usq;
        const R k = R(3) + R(9) * cu;
        a0 += l[i] * aw<R>(i) * P;
        bx += l[i] * aw<R>(i) * rho * (k * R(acx(i)) - R(3) * ux);
        by += l[i] * aw<R>(i) * rho * (k * R(acy(i)) - R(3) * uy);
    }
    const R it = R(1) / tau;
#pragma unroll
    for (int j = 0; j < 9; ++j)
        lam_out[L.at(j, y, x)] =
            (R(1) - it) * l[j] + it * (a0 + (bx * (R(acx(j)) - ux) + by * (R(acy(j)) - uy)) / rho);
}

template <typename R>
__global__ __launch_bounds__(kBlock) void adj_init_kernel(int nx, int ny, long long plane, PopLayout L,
                                                     const double* __restrict__ rho0,
                                                     const double* __restrict__ ux0,
                                                     const double* __restrict__ uy0,
                                                     const R* __restrict__ lam0,
                                                     double* __restrict__ gux,
                                                     double* __restrict__ guy)
{
    const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (c >= plane) return;
    const int x = (int)(c % nx), y = (int)(c / nx);
    R l[9];
    pull9<-1>(lam0, L, x, y, nx, ny, l);
    const double r = rho0[c], u = ux0[c], v = uy0[c];
    double gx = 0.0, gy = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const double cu = acx(i) * u + acy(i) * v;
        const double k = 3.0 + 9.0 * cu;
        const double wl = (double)l[i] * aw<double>(i) * r;
        gx += wl * (k * acx(i) - 3.0 * u);
        gy += wl * (k * acy(i) - 3.0 * v);
    }
    gux[c] = gx;
    guy[c] = gy;
}

static dim3 cells_grid(long long n) { return dim3((unsigned)((n + kBlock - 1) / kBlock)); }

hipError_t launch_adj_seed(int dtype, const D2Q9Args& a, const void* pop_prev, void* lam_out,
                           hipStream_t s)
{
    if (dtype == 0)
        adj_seed_kernel<double><<<cells_grid(a.plane), kBlock, 0, s>>>(
            a.nx, a.ny, a.plane, a.L, a.rho0, (const double*)pop_prev, (double*)lam_out);
    else if (dtype == 1)
        adj_seed_kernel<float><<<cells_grid(a.plane), kBlock, 0, s>>>(
            a.nx, a.ny, a.plane, a.L, (float)a.rho0, (const float*)pop_prev, (float*)lam_out);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_adj_step(int dtype, const D2Q9Args& a, const void* pop_prev, const void* lam_in,
                           void* lam_out, hipStream_t s)
{
    if (dtype == 0)
        adj_step_kernel<double><<<cells_grid(a.plane), kBlock, 0, s>>>(
            a.nx, a.ny, a.plane, a.L, a.rho0, a.tau, (const double*)pop_prev, (const double*)lam_in,
            (double*)lam_out);
    else if (dtype == 1)
        adj_step_kernel<float><<<cells_grid(a.plane), kBlock, 0, s>>>(
            a.nx, a.ny, a.plane, a.L, (float)a.rho0, (float)a.tau, (const float*)pop_prev,
            (const float*)lam_in, (float*)lam_out);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_adj_init(int dtype, const D2Q9Args& a, const double* rho0, const double* ux0,
                           const double* uy0, const void* lam0, double* gux, double* guy,
                           hipStream_t s)
{
    if (dtype == 0)
        adj_init_kernel<double><<<cells_grid(a.plane), kBlock, 0, s>>>(
            a.nx, a.ny, a.plane, a.L, rho0, ux0, uy0, (const double*)lam0, gux, guy);
    else if (dtype == 1)
        adj_init_kernel<float><<<cells_grid(a.plane), kBlock, 0, s>>>(
            a.nx, a.ny, a.plane, a.L, rho0, ux0, uy0, (const float*)lam0, gux, guy);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

} // namespace lks
