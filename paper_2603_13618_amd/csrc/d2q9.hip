// d2q9.hip -- D2Q9 lattice-BGK kernels for gfx950: the fused
// stream + collide + sensors + flags + FP64 sums pass, the three passes of the
// unfused baseline, the equilibrium initialiser and the moment readout.
//
// Method (arXiv 2603.13618): D2Q9 = GH3 x GH3 velocity set, order-2
// Grad-Hermite equilibrium (Sec. II.A.3), single-relaxation BGK (the QE
// collision of Sec. II.A.1 with tau1 = tau2), sensors S_KL (eq. HKL-sensor),
// S_NEQ (eq. sensor-neq-kin) and S_PI (eq. sensor-TauNS-kin) on the
// pre-collision populations, refinement flags (Sec. II.B.2, step 1).
//
// Memory layout: deviations d_i = f_i - w_i rho0, population i of cell (x, y)
// at i * pp + y * pr + x (PopLayout: plane-major [9][ny][nx] or
// row-interleaved [ny][9][nx], x fastest in both).  One thread owns VEC
// consecutive cells of a row, so every population row is read with one
// aligned VEC-wide load per thread; the x-shifted populations
// take their one missing neighbour from the adjacent lane (ds_bpermute) and
// only the wave's edge lanes touch memory for it.  Pull streaming reads each
// stored value exactly once, so HBM traffic is one read and one write per
// population plus the sensor planes and the flag byte.
#include "lks_device.h"
#include "lks_internal.h"

namespace lks {

// velocity i = 3a + b: c = (a - 1, b - 1); weights (1/6, 2/3, 1/6)^2
__device__ __forceinline__ constexpr int cx9(int i) { return i / 3 - 1; }
__device__ __forceinline__ constexpr int cy9(int i) { return i % 3 - 1; }
template <typename R>
__device__ __forceinline__ constexpr R w9(int i)
{
    return (i == 4) ? R(4.0 / 9.0) : ((cx9(i) == 0 || cy9(i) == 0) ? R(1.0 / 9.0) : R(1.0 / 36.0));
}

template <int N, typename F, int I = 0>
__device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<N, F, I + 1>(static_cast<F&&>(f));
    }
}

// Load VEC cells of row `row` starting at x0, shifted by cx along x
// (periodic): out[k] = row[(x0 + k - CX) mod nx].
template <int CX, typename S, int VEC>
__device__ __forceinline__ void pull_row(const typename Store<S>::raw* __restrict__ row, int x0,
                                         int nx, bool active, int lane,
                                         typename Store<S>::real (&out)[VEC])
{
    using R = typename Store<S>::real;
    R a[VEC];
    if (active) {
        load_vec<S, VEC>(row + x0, a);
    } else {
#pragma unroll
        for (int k = 0; k < VEC; ++k) a[k] = R(0);
    }
    if constexpr (CX == 0) {
#pragma unroll
        for (int k = 0; k < VEC; ++k) out[k] = a[k];
    } else if constexpr (CX == 1) {
        R prev = __shfl_up(a[VEC - 1], 1, kWave);
        if (active && (lane == 0 || x0 == 0))
            prev = Store<S>::to_real(row[x0 == 0 ? nx - 1 : x0 - 1]);
        out[0] = prev;
#pragma unroll
        for (int k = 1; k < VEC; ++k) out[k] = a[k - 1];
    } else {
        R next = __shfl_down(a[0], 1, kWave);
        if (active && (lane == kWave - 1 || x0 + VEC >= nx))
            next = Store<S>::to_real(row[x0 + VEC >= nx ? 0 : x0 + VEC]);
#pragma unroll
        for (int k = 0; k + 1 < VEC; ++k) out[k] = a[k + 1];
        out[VEC - 1] = next;
    }
}

// Per-cell result of the sensor part of the update.
template <typename R> struct CellSense {
    R kl, neq, pi;
    bool fault;
};

// One cell: moments, equilibrium, sensors and (if COLLIDE) the BGK collision
// of the pre-collision deviations d[0..8] in place.  EXT: also the extension
// sensors into ext[0..kNumExt) (mu = tau rho c_s^2, lambda = 0 on this
// isothermal lattice).
template <typename R, bool SENSE, bool COLLIDE, bool EXT = false>
__device__ __forceinline__ CellSense<R> cell_update(R (&d)[9], R rho0, R inv_tau, R& drho_out,
                                                    R& jx_out, R& jy_out, R* ext = nullptr,
                                                    unsigned ext_mask = 0)
{
    // moments of the deviation form: rho - rho0 = sum d, j = sum c d
    const R drho = ((d[0] + d[1]) + (d[2] + d[3])) + ((d[4] + d[5]) + (d[6] + d[7])) + d[8];
    const R jx = (d[6] + d[7] + d[8]) - (d[0] + d[1] + d[2]);
    const R jy = (d[2] + d[5] + d[8]) - (d[0] + d[3] + d[6]);
    const R rho = rho0 + drho;
    const R irho = rcp(rho);
    const R ux = jx * irho, uy = jy * irho;
    // f^eq_i - w_i rho0 = w_i [(rho - rho0) + rho (3 cu + 9/2 cu^2 - 3/2 u^2)]
    const R base = drho - R(1.5) * rho * (ux * ux + uy * uy);
    R deq[9];
    // corners c = (+-1, +-1)
#pragma unroll
    for (int i = 0; i < 9; i += 2) {
        if (i == 4) continue;
        const R cu = R(cx9(i)) * ux + R(cy9(i)) * uy;
        deq[i] = R(1.0 / 36.0) * (base + rho * (cu * (R(3) + R(4.5) * cu)));
    }
    // Axis pairs from their sum (even in u) and the momentum they must carry:
    // this closes sum_i c_i f^eq_i = j exactly up to the last rounding, so no
    // bias from the rounded weights is fed back by the collision.
    {
        const R sx = R(1.0 / 9.0) * (R(2) * base + R(9) * rho * ux * ux);
        const R dx = jx - ((deq[6] + deq[8]) - (deq[0] + deq[2]));
        deq[7] = R(0.5) * (sx + dx);
        deq[1] = R(0.5) * (sx - dx);
        const R sy = R(1.0 / 9.0) * (R(2) * base + R(9) * rho * uy * uy);
        const R dy = jy - ((deq[2] + deq[8]) - (deq[0] + deq[6]));
        deq[5] = R(0.5) * (sy + dy);
        deq[3] = R(0.5) * (sy - dy);
    }
    // rest population closes the mass
    deq[4] = drho - (((deq[0] + deq[1]) + (deq[2] + deq[3])) + ((deq[5] + deq[6]) + (deq[7] + deq[8])));

    CellSense<R> out{R(0), R(0), R(0), false};
    if constexpr (SENSE) {
        R kl = R(0), neq = R(0), pxx = R(0), pxy = R(0), pyy = R(0);
        R xmax = R(0), xmin = R(0), feqmin = R(0);
        bool far;
        {   // multiply-adds fuse within one expression only: the same bits in every kernel
#pragma clang fp contract(on)
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const R fneq = d[i] - deq[i];
                const R feq = w9<R>(i) * rho0 + deq[i];
                const R x = fneq * rcp(feq);
                // S_KL term feq phi(x) = fneq x p(x) on the series branch
                kl += (fneq * x) * kl_series_short(x);
                xmax = i == 0 ? fabs(x) : fmax(xmax, fabs(x));
                feqmin = i == 0 ? feq : fmin(feqmin, feq);
                neq += fabs(fneq);
                if (cx9(i) != 0) pxx += fneq;
                if (cy9(i) != 0) pyy += fneq;
                if (cx9(i) * cy9(i) != 0) pxy += R(cx9(i) * cy9(i)) * fneq;
            }
            // Rare: some population far from equilibrium (or NaN).  There the
            // smallest x is needed too (x > -1 is f > 0); on the short-series
            // branch |x| <= 0.03 already implies it.
            far = !(xmax <= KlShortCut<R>::v);
            if (far) {
                kl = R(0);
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    const R feq = w9<R>(i) * rho0 + deq[i];
                    const R x = (d[i] - deq[i]) * rcp(feq);
                    xmin = i == 0 ? x : fmin(xmin, x);
                    kl += feq * kl_phi(x);
                }
            }
        }
        out.fault = !(feqmin > R(0)) || (far && !(xmin > R(-1))) || !(kl == kl);
        out.kl = out.fault ? R(INFINITY) : kl;
        out.neq = neq;
        out.pi = sqrt_r(fma(pxx, pxx, fma(R(2) * pxy, pxy, pyy * pyy)));
        if constexpr (EXT) {
            // The extension sensors work on opaque copies (pin) of the
            // pre-collision deviations, their equilibrium parts and the
            // base quantities they need, and run after the collision: no
            // base expression gains a use and the base arithmetic stays in
            // one block, so its results do not depend on the extension.
            R dp[9], qp[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                dp[i] = pin(d[i]);
                qp[i] = pin(deq[i]);
            }
            const R kl_p = pin(kl), rho0_p = pin(rho0), tau_p = pin(inv_tau), irho_p = pin(irho);
            const R ux_p = pin(ux), uy_p = pin(uy);
            const R pxx_p = pin(pxx), pxy_p = pin(pxy), pyy_p = pin(pyy);
            const bool fault = out.fault;
            if constexpr (COLLIDE) {
#pragma unroll
                for (int i = 0; i < 9; ++i) d[i] -= inv_tau * (d[i] - deq[i]);
            }
            ExtAcc<R> xa;
            const ExtNeed need(ext_mask);
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const R fneq = dp[i] - qp[i];
                const R x = fneq * rcp(w9<R>(i) * rho0_p + qp[i]);
                // f = w rho0 + d; f^eq/w - 1 = (rho0 - 1) + deq/w
                xa.add(need, fneq, x, w9<R>(i) * rho0_p + dp[i],
                       (rho0_p - R(1)) + qp[i] * R(1.0 / w9<double>(i)));
            }
            R xv[kNumExt];
            const R inv_mu = R(3) * tau_p * irho_p;          // mu = tau rho / 3
            ext_finish<R>(xa, kl_p, fault, tau_p, inv_mu, pxx_p, pxy_p, pyy_p, ux_p, uy_p, R(0), R(0),
                          false, xv);
#pragma unroll
            for (int k = 0; k < kNumExt; ++k) ext[k] = xv[k];
            drho_out = drho;
            jx_out = jx;
            jy_out = jy;
            return out;
        }
    }
    if constexpr (COLLIDE) {
#pragma unroll
        for (int i = 0; i < 9; ++i) d[i] -= inv_tau * (d[i] - deq[i]);
    }
    drho_out = drho;
    jx_out = jx;
    jy_out = jy;
    return out;
}

template <typename S, int VEC, bool PULL>
__device__ __forceinline__ void load_row(const typename Store<S>::raw* __restrict__ fin, const PopLayout& L,
                                         int y, int nx, int ny, int x0, bool active, int lane,
                                         typename Store<S>::real (&d)[9][VEC])
{
    using R = typename Store<S>::real;
    static_for<9>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        constexpr int cx = PULL ? cx9(i) : 0;
        constexpr int cy = PULL ? cy9(i) : 0;
        int ys = y - cy;
        ys = ys < 0 ? ys + ny : (ys >= ny ? ys - ny : ys);
        R v[VEC];
        pull_row<cx, S, VEC>(fin + L.at(i, ys, 0), x0, nx, active, lane, v);
#pragma unroll
        for (int k = 0; k < VEC; ++k) d[i][k] = v[k];
    });
}

// One workgroup: `rows` consecutive rows of one x-tile.  The next row's
// populations are loaded before the current row is computed, so each wave
// keeps a row of loads in flight behind its arithmetic.
template <typename S, int VEC, int PASS>
__global__ __launch_bounds__(kBlock) LKS_CELL_KERNEL_ATTR void d2q9_kernel(
    D2Q9Args a, const typename Store<S>::raw* __restrict__ fin, typename Store<S>::raw* __restrict__ fout,
    typename Store<S>::real* __restrict__ sens, uint8_t* __restrict__ flags,
    double* __restrict__ partials, unsigned long long* __restrict__ faults)
{
    using R = typename Store<S>::real;
    constexpr bool PULL = (PASS == kFused || PASS == kStream);
    constexpr bool SENSE = (PASS == kFused || PASS == kSense);
    constexpr bool COLLIDE = (PASS == kFused || PASS == kCollide);

    const int nx = a.nx, ny = a.ny;
    const long long plane = a.plane;
    const int lane = threadIdx.x & (kWave - 1);
    const int tx = blockIdx.x % a.g.tiles_x;
    const int rg = blockIdx.x / a.g.tiles_x;
    const int x0 = (tx * kBlock + threadIdx.x) * VEC;
    const bool active = x0 < nx;
    const int y0 = rg * a.g.rows;
    const int y1 = min(y0 + a.g.rows, ny);

    constexpr bool F32 = sizeof(R) == 4;
    const R rho0 = F32 ? R(a.rho0_f) : R(a.rho0);
    const R inv_tau = F32 ? R(a.inv_tau_f) : R(1.0 / a.tau);
    R th[3][2];
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        th[s][0] = F32 ? R(a.thr_f[s][0]) : R(a.thr[s][0]);
        th[s][1] = F32 ? R(a.thr_f[s][1]) : R(a.thr[s][1]);
    }
    double acc[kNsums];
#pragma unroll
    for (int k = 0; k < kNsums; ++k) acc[k] = 0.0;
    unsigned nfault = 0;

    // ring of PF + 1 rows: rows y .. y + PF - 1 are loaded or in flight while
    // row y is computed
    constexpr int PF = LKS_D2Q9_PREFETCH;
    R ring[PF + 1][9][VEC];
#pragma unroll
    for (int p = 0; p < PF; ++p)
        if (y0 + p < y1) load_row<S, VEC, PULL>(fin, a.L, y0 + p, nx, ny, x0, active, lane, ring[p]);
    for (int y = y0; y < y1; ++y) {                 // uniform across the workgroup
        if (y + PF < y1) load_row<S, VEC, PULL>(fin, a.L, y + PF, nx, ny, x0, active, lane, ring[PF]);
        R (&cur)[9][VEC] = ring[0];
        const long long off = (long long)y * nx + x0;
        const long long poff = a.L.at(0, y, x0);

        if constexpr (PASS == kStream) {
            if (active) {
#pragma unroll
                for (int i = 0; i < 9; ++i) store_vec<S, VEC>(fout + i * a.L.pp + poff, cur[i]);
            }
        } else {
            R s_kl[VEC], s_neq[VEC], s_pi[VEC];
            uint8_t fl[VEC];
#pragma unroll
            for (int k = 0; k < VEC; ++k) {
                R dc[9];
#pragma unroll
                for (int i = 0; i < 9; ++i) dc[i] = cur[i][k];
                R drho, jx, jy;
                LKS_CELL_BARRIER();
                const CellSense<R> cs = cell_update<R, SENSE, COLLIDE>(dc, rho0, inv_tau, drho, jx, jy);
#pragma unroll
                for (int i = 0; i < 9; ++i) cur[i][k] = dc[i];
                if constexpr (SENSE) {
                    LevelAcc lv;
                    const R sv[3] = {cs.kl, cs.neq, cs.pi};
#pragma unroll
                    for (int s = 0; s < 3; ++s) lv.add(sv[s], th[s][0], th[s][1]);
                    fl[k] = cs.fault ? uint8_t(0x82) : uint8_t(lv.level());
                    s_kl[k] = cs.kl;
                    s_neq[k] = cs.neq;
                    s_pi[k] = cs.pi;
                    if (active) {
                        // each cell's terms widen to FP64 before any add: FP64
                        // sums of FP32 values do not depend on the grouping,
                        // i.e. on the launch shape
                        acc[0] += (double)drho;
                        acc[1] += (double)jx;
                        acc[2] += (double)jy;
                        acc[4] += (double)cs.kl;
                        acc[5] += (double)cs.neq;
                        acc[6] += (double)cs.pi;
                        nfault += cs.fault ? 1u : 0u;
                    }
                }
            }
            if (active) {
                if constexpr (COLLIDE) {
#pragma unroll
                    for (int i = 0; i < 9; ++i) store_vec<S, VEC>(fout + i * a.L.pp + poff, cur[i]);
                }
                if constexpr (SENSE) {
                    store_pack<R, VEC>(sens + off, s_kl);
                    store_pack<R, VEC>(sens + plane + off, s_neq);
                    store_pack<R, VEC>(sens + 2 * plane + off, s_pi);
                    store_pack<uint8_t, VEC>(flags + off, fl);
                }
            }
        }
#pragma unroll
        for (int p = 0; p < PF; ++p)
#pragma unroll
            for (int i = 0; i < 9; ++i)
#pragma unroll
                for (int k = 0; k < VEC; ++k) ring[p][i][k] = ring[p + 1][i][k];
    }
    if constexpr (SENSE) {
        if (nfault) atomicAdd(faults, (unsigned long long)nfault);
        block_sums(acc, partials + (long long)blockIdx.x * kNsums);
    }
}

// Fused step with the next row staged through LDS by direct global->LDS
// loads: the row in flight occupies no registers.  Each wave owns a private
// 9 x 1 KB staging area.  A lane's VEC cells of population i are CHUNK bytes;
// they arrive in NP pieces of PS bytes (the direct loads move 1, 2, 4, 12 or
// 16 bytes per lane), piece p of lane l at i*1024 + p*64*PS + l*PS, and are
// read back by the same lane.
// how a lane's VEC cells of one population travel through the staging area
template <typename S, int VEC> struct StageGeom {
    static constexpr int CHUNK = VEC * (int)sizeof(typename Store<S>::raw);
    static constexpr int NP0 = CHUNK == 8 ? 2 : 1;
    static constexpr int PS0 = CHUNK / NP0;
    static constexpr int PE0 = PS0 / (int)sizeof(typename Store<S>::raw);
    // usable when every piece holds whole elements and is a whole number of
    // dwords: a sub-dword direct load writes lane l's value into the 4-byte
    // LDS slot l, not at (piece size) x l, so 1- and 2-byte pieces would not
    // land contiguously
    static constexpr bool ok = PE0 >= 1 && (PS0 == 4 || PS0 == 16);
    // (a geometry that is not ok is never launched; keep it compilable)
    static constexpr int NP = ok ? NP0 : 1;           // pieces per lane
    static constexpr int PS = ok ? PS0 : 4;           // bytes per piece
    static constexpr int PE = ok ? PE0 : 1;           // elements per piece
};

// NT: stores with the non-temporal hint (the launcher sets it when the two
// state buffers exceed the last-level cache, so the next step's loads come
// from HBM anyway)
template <typename S, int VEC, bool EXT = false, bool NT = false>
__global__ __launch_bounds__(kBlock) LKS_CELL_KERNEL_ATTR void d2q9_fused_lds(
    D2Q9Args a, const typename Store<S>::raw* __restrict__ fin, typename Store<S>::raw* __restrict__ fout,
    typename Store<S>::real* __restrict__ sens, uint8_t* __restrict__ flags,
    double* __restrict__ partials, unsigned long long* __restrict__ faults)
{
    using R = typename Store<S>::real;
    using raw = typename Store<S>::raw;
    using G = StageGeom<S, VEC>;
    typedef __attribute__((address_space(1))) void gvoid;
    typedef __attribute__((address_space(3))) void lvoid;
    // per wave: one row of the nine planes, and for each x-shifted plane the
    // one value just outside the wave's span of cells
    __shared__ __attribute__((aligned(16))) unsigned char stage[kBlock / kWave][9][1024];
    __shared__ __attribute__((aligned(16))) unsigned char halo[kBlock / kWave][9][8];
    constexpr int ES = (int)sizeof(raw);        // bytes per element
    constexpr int EP = ES < 4 ? ES : 4;         // bytes per direct-load piece of an edge value
    constexpr int NEP = ES / EP;                // pieces per edge value

    const int nx = a.nx, ny = a.ny;
    const long long plane = a.plane;
    const int lane = threadIdx.x & (kWave - 1);
    // 16-bit storage (VALU-bound): the wave index taken wave-uniform, so the
    // staging area's LDS addresses are scalar, and row accesses as a uniform
    // row base plus a 32-bit lane offset (BF16 at 8192^2 649 -> 639 us; the
    // same forms made FP32 3 % slower, which keeps the plain ones)
    constexpr bool kHalf = sizeof(raw) == 2;
    const int wave = kHalf ? __builtin_amdgcn_readfirstlane(threadIdx.x / kWave) : threadIdx.x / kWave;
    const int tx = blockIdx.x % a.g.tiles_x;
    const int rg = blockIdx.x / a.g.tiles_x;
    const int x0 = (tx * kBlock + threadIdx.x) * VEC;
    const bool active = x0 < nx;
    const int y0 = rg * a.g.rows;
    const int y1 = min(y0 + a.g.rows, ny);
    // the wave's span of cells and its periodic neighbours (nx % VEC == 0)
    const int xw = (tx * kBlock + wave * kWave) * VEC;
    const bool wave_active = xw < nx;
    const int xl = xw == 0 ? nx - 1 : xw - 1;
    const int xr = xw + kWave * VEC >= nx ? 0 : xw + kWave * VEC;
    const bool last_lane = lane == kWave - 1 || x0 + VEC >= nx;

    constexpr bool F32 = sizeof(R) == 4;
    const R rho0 = F32 ? R(a.rho0_f) : R(a.rho0);
    const R inv_tau = F32 ? R(a.inv_tau_f) : R(1.0 / a.tau);
    R th[3][2];
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        th[s][0] = F32 ? R(a.thr_f[s][0]) : R(a.thr[s][0]);
        th[s][1] = F32 ? R(a.thr_f[s][1]) : R(a.thr[s][1]);
    }
    double acc[kNsums];
#pragma unroll
    for (int k = 0; k < kNsums; ++k) acc[k] = 0.0;
    unsigned nfault = 0;

    // Row y of every plane into this wave's staging area.  Only direct
    // global->LDS loads: no register results, so nothing here makes the
    // wave wait for the loads it has just issued.
    auto issue = [&](int y) {
        static_for<9>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            constexpr int cx = cx9(i), cy = cy9(i);
            int ys = y - cy;
            ys = ys < 0 ? ys + ny : (ys >= ny ? ys - ny : ys);
            const raw* row = fin + a.L.at(i, ys, 0);
            if (active) {
#pragma unroll
                for (int p = 0; p < G::NP; ++p) {
                    gvoid* g = kHalf ? (gvoid*)(row + (unsigned)(x0 + p * G::PE)) : (gvoid*)(row + x0 + p * G::PE);
                    lvoid* l = (lvoid*)&stage[wave][i][p * kWave * G::PS];
                    if constexpr (G::PS == 16) __builtin_amdgcn_global_load_lds(g, l, 16, 0, 0);
                    else __builtin_amdgcn_global_load_lds(g, l, 4, 0, 0);
                }
            }
            if constexpr (cx != 0) {
                // lanes 0 .. NEP-1 fetch the pieces of the edge value (for a
                // 16-bit value only lane 0, whose LDS slot starts at offset 0)
                if (wave_active && lane < NEP) {
                    const int xe = cx == 1 ? xl : xr;
                    gvoid* g = (gvoid*)(reinterpret_cast<const unsigned char*>(row + xe) + lane * EP);
                    lvoid* l = (lvoid*)&halo[wave][i][0];
                    if constexpr (EP == 4) __builtin_amdgcn_global_load_lds(g, l, 4, 0, 0);
                    else if constexpr (EP == 2) __builtin_amdgcn_global_load_lds(g, l, 2, 0, 0);
                    else __builtin_amdgcn_global_load_lds(g, l, 1, 0, 0);
                }
            }
        });
    };

    // results of one row, stored while the next row computes
    R res[9][VEC];
    R s_kl[VEC], s_neq[VEC], s_pi[VEC];
    uint8_t fl[VEC];
    R xres[EXT ? kNumExt : 1][VEC];
    auto store_row = [&](int y) {
        if (active) {
            const long long off = (long long)y * nx + x0;
            if constexpr (kHalf) {
                const unsigned ux = (unsigned)x0;
                const long long srow = (long long)y * nx, prow = a.L.at(0, y, 0);
#pragma unroll
                for (int i = 0; i < 9; ++i) store_vec<S, VEC, NT>(fout + (i * a.L.pp + prow) + ux, res[i]);
                store_pack<R, VEC, NT>(sens + srow + ux, s_kl);
                store_pack<R, VEC, NT>(sens + (plane + srow) + ux, s_neq);
                store_pack<R, VEC, NT>(sens + (2 * plane + srow) + ux, s_pi);
                store_pack<uint8_t, VEC, NT>(flags + srow + ux, fl);
            } else {
                const long long poff = a.L.at(0, y, x0);
#pragma unroll
                for (int i = 0; i < 9; ++i) store_vec<S, VEC, NT>(fout + i * a.L.pp + poff, res[i]);
                store_pack<R, VEC, NT>(sens + off, s_kl);
                store_pack<R, VEC, NT>(sens + plane + off, s_neq);
                store_pack<R, VEC, NT>(sens + 2 * plane + off, s_pi);
                store_pack<uint8_t, VEC, NT>(flags + off, fl);
            }
            if constexpr (EXT) {
#pragma unroll
                for (int q = 0; q < kNumExt; ++q)
                    if (a.x.plane[q] >= 0) store_pack<R, VEC, NT>(sens + a.x.plane[q] * plane + off, xres[q]);
            }
        }
    };

    if (y0 < y1) issue(y0);
    for (int y = y0; y < y1; ++y) {                 // uniform across the workgroup
        // row y has landed in LDS (and the stores of row y - 2 have completed)
        wait_vmem_all();
        R cur[9][VEC];
        static_for<9>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            constexpr int cx = cx9(i);
            R v[VEC];
#pragma unroll
            for (int p = 0; p < G::NP; ++p) {
                R piece[G::PE];
                load_vec<S, G::PE>(reinterpret_cast<const raw*>(
                                       &stage[wave][i][p * kWave * G::PS + lane * G::PS]), piece);
#pragma unroll
                for (int k = 0; k < G::PE; ++k) v[p * G::PE + k] = piece[k];
            }
            if constexpr (cx == 0) {
#pragma unroll
                for (int k = 0; k < VEC; ++k) cur[i][k] = v[k];
            } else {
                const R e = Store<S>::to_real(*reinterpret_cast<const raw*>(&halo[wave][i][0]));
                if constexpr (cx == 1) {
                    const R prev = __shfl_up(v[VEC - 1], 1, kWave);
                    cur[i][0] = lane == 0 ? e : prev;
#pragma unroll
                    for (int k = 1; k < VEC; ++k) cur[i][k] = v[k - 1];
                } else {
                    const R next = __shfl_down(v[0], 1, kWave);
#pragma unroll
                    for (int k = 0; k + 1 < VEC; ++k) cur[i][k] = v[k + 1];
                    cur[i][VEC - 1] = last_lane ? e : next;
                }
            }
        });
        // the staging area is rewritten by the next row's loads only after
        // every lane's reads of this row have completed
        wait_lds_all();
        if (y + 1 < y1) issue(y + 1);
        // the previous row's stores go out after the next row's loads, so
        // the wait for those loads at the top of the next iteration has this
        // row's whole computation to cover both (stores count in vmcnt too)
        if (y > y0) store_row(y - 1);

#pragma unroll
        for (int k = 0; k < VEC; ++k) {
            R dc[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) dc[i] = cur[i][k];
            R drho, jx, jy;
            R xv[kNumExt];
            LKS_CELL_BARRIER();
            const CellSense<R> cs = cell_update<R, true, true, EXT>(dc, rho0, inv_tau, drho, jx, jy, xv,
                                                                    a.x.mask);
#pragma unroll
            for (int i = 0; i < 9; ++i) res[i][k] = dc[i];
            LevelAcc lv;
            const R sv[3] = {cs.kl, cs.neq, cs.pi};
#pragma unroll
            for (int s = 0; s < 3; ++s) lv.add(sv[s], th[s][0], th[s][1]);
            if constexpr (EXT) {
#pragma unroll
                for (int q = 0; q < kNumExt; ++q) {
                    xres[q][k] = xv[q];
                    if (a.mask & (1u << (kExtFlagShift + q))) {
                        const R t0 = F32 ? R(a.x.thr_f[q][0]) : R(a.x.thr[q][0]);
                        const R t1 = F32 ? R(a.x.thr_f[q][1]) : R(a.x.thr[q][1]);
                        lv.add(xv[q], t0, t1);
                    }
                }
            }
            fl[k] = cs.fault ? uint8_t(0x82) : uint8_t(lv.level());
            s_kl[k] = cs.kl;
            s_neq[k] = cs.neq;
            s_pi[k] = cs.pi;
            if (active) {
                // each cell's terms widen to FP64 before any add (as above)
                acc[0] += (double)drho;
                acc[1] += (double)jx;
                acc[2] += (double)jy;
                acc[4] += (double)cs.kl;
                acc[5] += (double)cs.neq;
                acc[6] += (double)cs.pi;
                nfault += cs.fault ? 1u : 0u;
            }
        }
    }
    if (y0 < y1) store_row(y1 - 1);
    if (nfault) atomicAdd(faults, (unsigned long long)nfault);
    block_sums(acc, partials + (long long)blockIdx.x * kNsums);
}

// Two fused steps per pass over HBM (temporal blocking): the API keeps
// only the last step's sensors and flags, so a wave can advance its cells two
// steps from one read of the state.  Each wave owns a strip of kSweepW = 60
// columns and kSweepH rows: its 64 lanes hold the strip and a two-column ring
// (periodic), one column per lane, and the wave sweeps down the rows with its
// state in registers.  Raw row q arrives; step A runs on row q - 1 (lanes 1 to
// 62: the strip and a one-column ring), with the x neighbours from the
// adjacent lanes (DPP wave shifts) and the y neighbours from the two previous
// raw rows; its post-collision values, rounded to the storage type as a stored
// state would be, feed step B in the same way.  Step B runs on row q - 3
// (lanes 2 to 61) from step-A rows of earlier iterations, so the two cell
// updates of an iteration are independent and their instructions interleave.
// The strip's rows plus a two-row ring are read once; step B stores
// populations, sensors and flags.  No LDS and no barrier until the final sums.
// Each cell's sums and faults are counted by the wave that owns it, for both
// steps.  The loads of raw rows q + 1 and q + 2 are in flight while row q is
// used.  kSweepH = 16 rows per wave: short strips give more independent waves,
// which hides latency better than the shorter ring of tall strips saves bytes.
// Each cell's arithmetic is cell_update, as in the one-step kernels, so the
// results are bit-identical to two one-step launches.  A step that has no
// partner (an odd batch end) runs in the one-step kernel: this sweep with a
// single step measured 362.8 against 233.2 us at 4096^2.
constexpr int kSweepW = kWave - 4;
constexpr int kSweepH = 16;

// Periodic index for j in [-2, n + 1] (exact for n >= 2; n = 1 maps every j
// to 0).  Indexes further out only feed cells that are not stored: any
// in-range index serves them, so they are clamped.
__device__ __forceinline__ int wrap_index(int j, int n)
{
    j += j < 0 ? n : 0;
    j -= j >= n ? n : 0;
    return min(max(j, 0), n - 1);
}

// The value of lane l - CX (CX = +1: from the lane below, -1: from the lane
// above); lanes whose source is outside the wave get 0.
template <int CX>
__device__ __forceinline__ float lane_shift(float v)
{
    if constexpr (CX == 0) {
        return v;
    } else {
        constexpr int ctrl = CX > 0 ? 0x138 : 0x130;    // wave_shr:1 / wave_shl:1
        return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), ctrl,
                                                                     0xf, 0xf, false));
    }
}
template <int CX>
__device__ __forceinline__ double lane_shift(double v)
{
    if constexpr (CX == 0) {
        return v;
    } else {
        const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
        const float lo = lane_shift<CX>(__builtin_bit_cast(float, (unsigned)u));
        const float hi = lane_shift<CX>(__builtin_bit_cast(float, (unsigned)(u >> 32)));
        return __builtin_bit_cast(double, (unsigned long long)__builtin_bit_cast(unsigned, lo) |
                                              ((unsigned long long)__builtin_bit_cast(unsigned, hi) << 32));
    }
}

// Pre-step values of a cell at row y: population i from row y - cy_i (prev2,
// prev, cur for cy = +1, 0, -1) and lane l - cx_i.
template <typename R>
__device__ __forceinline__ void gather_pull(R (&d)[9], const R (&prev2)[9], const R (&prev)[9], const R (&cur)[9])
{
    static_for<9>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        constexpr int cy = cy9(i), cx = cx9(i);
        const R v = cy > 0 ? prev2[i] : (cy == 0 ? prev[i] : cur[i]);
        d[i] = lane_shift<cx>(v);
    });
}

template <typename S>
__global__ __launch_bounds__(kBlock) void d2q9_fused2_kernel(
    D2Q9Args a, const typename Store<S>::raw* __restrict__ fin, typename Store<S>::raw* __restrict__ fout,
    typename Store<S>::real* __restrict__ sens, uint8_t* __restrict__ flags, double* __restrict__ part_a,
    double* __restrict__ part_b, unsigned long long* __restrict__ faults)
{
    using R = typename Store<S>::real;
    const int nx = a.nx, ny = a.ny;
    const long long plane = a.plane;
    const int lane = threadIdx.x & (kWave - 1);
    const int strips = (nx + kSweepW - 1) / kSweepW, segs = (ny + kSweepH - 1) / kSweepH;
    const int wid = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    const bool has = wid < strips * segs;
    const int X0 = (wid % strips) * kSweepW, Yb = (wid / strips) * kSweepH;
    const int Ye = min(Yb + kSweepH, ny);
    const int X = X0 - 2 + lane;                  // this lane's column
    const int gx = wrap_index(X, nx);
    const bool own_col = lane >= 2 && lane < kSweepW + 2 && X < nx;

    constexpr bool F32 = sizeof(R) == 4;
    const R rho0 = F32 ? R(a.rho0_f) : R(a.rho0);
    const R inv_tau = F32 ? R(a.inv_tau_f) : R(1.0 / a.tau);
    R th[3][2];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        th[k][0] = F32 ? R(a.thr_f[k][0]) : R(a.thr[k][0]);
        th[k][1] = F32 ? R(a.thr_f[k][1]) : R(a.thr[k][1]);
    }
    auto level_of = [&](const CellSense<R>& cs) {
        LevelAcc lv;
        const R sv[3] = {cs.kl, cs.neq, cs.pi};
#pragma unroll
        for (int k = 0; k < 3; ++k) lv.add(sv[k], th[k][0], th[k][1]);
        return cs.fault ? uint8_t(0x82) : uint8_t(lv.level());
    };
    auto store_cell = [&](int Y, const R (&d)[9], const CellSense<R>& cs) {
        const long long off = (long long)Y * nx + X;
#pragma unroll
        for (int i = 0; i < 9; ++i) fout[a.L.at(i, Y, X)] = Store<S>::from_real(d[i]);
        sens[off] = cs.kl;
        sens[plane + off] = cs.neq;
        sens[2 * plane + off] = cs.pi;
        flags[off] = level_of(cs);
    };
    auto add_sums = [&](double (&acc)[kNsums], unsigned& nf, R drho, R jx, R jy, const CellSense<R>& cs) {
        acc[0] += (double)drho;
        acc[1] += (double)jx;
        acc[2] += (double)jy;
        acc[4] += (double)cs.kl;
        acc[5] += (double)cs.neq;
        acc[6] += (double)cs.pi;
        nf += cs.fault ? 1u : 0u;
    };
    auto load_row = [&](int q, R (&r)[9]) {
        const int gy = wrap_index(q, ny);
#pragma unroll
        for (int i = 0; i < 9; ++i) r[i] = Store<S>::to_real(fin[a.L.at(i, gy, gx)]);
    };

    double acc_a[kNsums], acc_b[kNsums];
#pragma unroll
    for (int k = 0; k < kNsums; ++k) acc_a[k] = acc_b[k] = 0.0;
    unsigned nfault = 0;

    if (has) {
        // raw rows qs .. qe; step A on rows qs + 1 .. qe - 1, step B on Yb .. Ye - 1
        const int qs = Yb - 2, qe = Ye + 1;
        R prev2[9], prev[9], cur[9], nxt[9] = {}, nxt2[9] = {};
        R aprev3[9], aprev2[9], aprev[9];
        load_row(qs, prev2);
        load_row(qs + 1, prev);
        load_row(qs + 2, cur);
        if (qs + 3 <= qe) load_row(qs + 3, nxt);
        const int qend = qe + 1;
        for (int q = qs + 2; q <= qend; ++q) {
            if (q + 2 <= qe) load_row(q + 2, nxt2);
            // ---- step B on row q - 3 (step A rows q - 4, q - 3, q - 2 of earlier iterations)
            if (q >= qs + 5) {
                R e[9];
                gather_pull(e, aprev3, aprev2, aprev);
                R drho2, jx2, jy2;
                const CellSense<R> cs2 = cell_update<R, true, true>(e, rho0, inv_tau, drho2, jx2, jy2);
                if (own_col) {
                    store_cell(q - 3, e, cs2);
                    add_sums(acc_b, nfault, drho2, jx2, jy2, cs2);
                }
            }
            if (q <= qe) {
                const int ya = q - 1;
                R d[9];
                gather_pull(d, prev2, prev, cur);
                R drho, jx, jy;
                const CellSense<R> cs = cell_update<R, true, true>(d, rho0, inv_tau, drho, jx, jy);
                const bool own_a = own_col && ya >= Yb && ya < Ye;
                if (own_a) add_sums(acc_a, nfault, drho, jx, jy, cs);
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    aprev3[i] = aprev2[i];
                    aprev2[i] = aprev[i];
                    aprev[i] = Store<S>::to_real(Store<S>::from_real(d[i]));
                }
            }
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                prev2[i] = prev[i];
                prev[i] = cur[i];
                cur[i] = nxt[i];
                nxt[i] = nxt2[i];
            }
        }
    }
    block_sums(acc_a, part_a + (long long)blockIdx.x * kNsums);
    __syncthreads();                              // block_sums' LDS is read before it is written again
    block_sums(acc_b, part_b + (long long)blockIdx.x * kNsums);
    if (nfault) atomicAdd(faults, (unsigned long long)nfault);
}

template <typename S>
static hipError_t launch_two(const D2Q9Args& a, const void* fin, void* fout, void* sens, uint8_t* flags,
                             double* part_a, double* part_b, unsigned long long* faults, hipStream_t st)
{
    using raw = typename Store<S>::raw;
    using R = typename Store<S>::real;
    const dim3 grid((unsigned)d2q9_two_blocks(sizeof(raw) == 8 ? 0 : 1, a.nx, a.ny)), block(kBlock);
    d2q9_fused2_kernel<S><<<grid, block, 0, st>>>(a, (const raw*)fin, (raw*)fout, (R*)sens, flags, part_a,
                                                  part_b, faults);
    return hipGetLastError();
}

// Workgroups of the two-step launches: one wave per strip of kSweepW columns
// and kSweepH rows.
int d2q9_two_blocks(int dtype, int nx, int ny)
{
    (void)dtype;
    const long long waves = (long long)((nx + kSweepW - 1) / kSweepW) * ((ny + kSweepH - 1) / kSweepH);
    return (int)((waves + kBlock / kWave - 1) / (kBlock / kWave));
}

hipError_t launch_d2q9_two(int dtype, const D2Q9Args& a, const void* fin, void* fout, void* sens,
                           uint8_t* flags, double* part_a, double* part_b, unsigned long long* faults,
                           hipStream_t s)
{
    switch (dtype) {
    case 0: return launch_two<double>(a, fin, fout, sens, flags, part_a, part_b, faults, s);
    case 1: return launch_two<float>(a, fin, fout, sens, flags, part_a, part_b, faults, s);
    case 2: return launch_two<bf16_t>(a, fin, fout, sens, flags, part_a, part_b, faults, s);
    case 3: return launch_two<f16_t>(a, fin, fout, sens, flags, part_a, part_b, faults, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename S, int VEC>
static hipError_t launch_pass(int pass, const D2Q9Args& a, const void* fin, void* fout, void* sens,
                              uint8_t* flags, double* partials, unsigned long long* faults,
                              hipStream_t st)
{
    using raw = typename Store<S>::raw;
    using R = typename Store<S>::real;
    const raw* in = static_cast<const raw*>(fin);
    raw* out = static_cast<raw*>(fout);
    R* sv = static_cast<R*>(sens);
    const dim3 grid(a.g.nblocks), block(kBlock);
    switch (pass) {
    case kFused:
        if (a.x.mask) {
            // extension sensors: F32 and F64 storage, whose pieces always stage
            if constexpr (std::is_same<S, float>::value || std::is_same<S, double>::value) {
                if (!(LKS_D2Q9_LDS_STAGE && StageGeom<S, VEC>::ok)) return hipErrorInvalidValue;
                d2q9_fused_lds<S, VEC, true><<<grid, block, 0, st>>>(a, in, out, sv, flags, partials, faults);
            } else {
                return hipErrorInvalidValue;
            }
        } else if (LKS_D2Q9_LDS_STAGE && StageGeom<S, VEC>::ok && a.nt_stores)
            d2q9_fused_lds<S, VEC, false, true><<<grid, block, 0, st>>>(a, in, out, sv, flags, partials, faults);
        else if (LKS_D2Q9_LDS_STAGE && StageGeom<S, VEC>::ok)
            d2q9_fused_lds<S, VEC><<<grid, block, 0, st>>>(a, in, out, sv, flags, partials, faults);
        else
            d2q9_kernel<S, VEC, kFused><<<grid, block, 0, st>>>(a, in, out, sv, flags, partials, faults);
        break;
    case kStream:
        d2q9_kernel<S, VEC, kStream><<<grid, block, 0, st>>>(a, in, out, sv, flags, partials, faults);
        break;
    case kSense:
        d2q9_kernel<S, VEC, kSense><<<grid, block, 0, st>>>(a, in, out, sv, flags, partials, faults);
        break;
    case kCollide:
        d2q9_kernel<S, VEC, kCollide><<<grid, block, 0, st>>>(a, in, out, sv, flags, partials, faults);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename S, int VWIDE>
static hipError_t launch_vec(int pass, const D2Q9Args& a, const void* fin, void* fout, void* sens,
                             uint8_t* flags, double* partials, unsigned long long* faults,
                             hipStream_t st)
{
    switch (a.g.vec) {
    case 1: return launch_pass<S, 1>(pass, a, fin, fout, sens, flags, partials, faults, st);
    case 2: return launch_pass<S, 2>(pass, a, fin, fout, sens, flags, partials, faults, st);
    case 4:
        if constexpr (VWIDE >= 4) return launch_pass<S, 4>(pass, a, fin, fout, sens, flags, partials, faults, st);
        return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_d2q9(int dtype, int pass, const D2Q9Args& a, const void* fin, void* fout,
                       void* sens, uint8_t* flags, double* partials, unsigned long long* faults,
                       hipStream_t s)
{
    switch (dtype) {
    case 0: return launch_vec<double, 2>(pass, a, fin, fout, sens, flags, partials, faults, s);
    case 1: return launch_vec<float, 4>(pass, a, fin, fout, sens, flags, partials, faults, s);
    case 2: return launch_vec<bf16_t, 4>(pass, a, fin, fout, sens, flags, partials, faults, s);
    case 3: return launch_vec<f16_t, 4>(pass, a, fin, fout, sens, flags, partials, faults, s);
    default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// Equilibrium initialiser and moment readout (one thread per cell, FP64 math)
// ---------------------------------------------------------------------------
template <typename S>
__global__ __launch_bounds__(kBlock) void d2q9_init_kernel(long long n, PopLayout L, double rho0, const double* __restrict__ rho,
                                                      const double* __restrict__ ux,
                                                      const double* __restrict__ uy,
                                                      typename Store<S>::raw* __restrict__ pop)
{
    const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (c >= n) return;
    const double r = rho[c], u = ux[c], v = uy[c];
    const double usq15 = 1.5 * (u * u + v * v);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const double cu = cx9(i) * u + cy9(i) * v;
        const double deq = w9<double>(i) * ((r - rho0) + r * (cu * (3.0 + 4.5 * cu) - usq15));
        pop[L.cell(i, c)] = Store<S>::from_real((typename Store<S>::real)deq);
    }
}

template <typename S>
__global__ __launch_bounds__(kBlock) void d2q9_moments_kernel(long long n, PopLayout L, double rho0,
                                                         const typename Store<S>::raw* __restrict__ pop,
                                                         double* __restrict__ rho, double* __restrict__ ux,
                                                         double* __restrict__ uy, double* __restrict__ T)
{
    const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (c >= n) return;
    double drho = 0.0, jx = 0.0, jy = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const double d = (double)Store<S>::to_real(pop[L.cell(i, c)]);
        drho += d;
        jx += cx9(i) * d;
        jy += cy9(i) * d;
    }
    const double r = rho0 + drho;
    rho[c] = r;
    ux[c] = jx / r;
    uy[c] = jy / r;
    if (T) T[c] = 1.0 / 3.0;
}

hipError_t launch_d2q9_init(int dtype, long long n, const PopLayout& L, double rho0, const double* rho,
                            const double* ux, const double* uy, void* pop, hipStream_t s)
{
    const dim3 grid((unsigned)((n + kBlock - 1) / kBlock)), block(kBlock);
    switch (dtype) {
    case 0: d2q9_init_kernel<double><<<grid, block, 0, s>>>(n, L, rho0, rho, ux, uy, (double*)pop); break;
    case 1: d2q9_init_kernel<float><<<grid, block, 0, s>>>(n, L, rho0, rho, ux, uy, (float*)pop); break;
    case 2: d2q9_init_kernel<bf16_t><<<grid, block, 0, s>>>(n, L, rho0, rho, ux, uy, (uint16_t*)pop); break;
    case 3: d2q9_init_kernel<f16_t><<<grid, block, 0, s>>>(n, L, rho0, rho, ux, uy, (uint16_t*)pop); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_d2q9_moments(int dtype, long long n, const PopLayout& L, double rho0, const void* pop,
                               double* rho, double* ux, double* uy, double* T, hipStream_t s)
{
    const dim3 grid((unsigned)((n + kBlock - 1) / kBlock)), block(kBlock);
    switch (dtype) {
    case 0: d2q9_moments_kernel<double><<<grid, block, 0, s>>>(n, L, rho0, (const double*)pop, rho, ux, uy, T); break;
    case 1: d2q9_moments_kernel<float><<<grid, block, 0, s>>>(n, L, rho0, (const float*)pop, rho, ux, uy, T); break;
    case 2: d2q9_moments_kernel<bf16_t><<<grid, block, 0, s>>>(n, L, rho0, (const uint16_t*)pop, rho, ux, uy, T); break;
    case 3: d2q9_moments_kernel<f16_t><<<grid, block, 0, s>>>(n, L, rho0, (const uint16_t*)pop, rho, ux, uy, T); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

} // namespace lks
