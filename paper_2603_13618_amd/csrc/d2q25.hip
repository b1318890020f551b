// d2q25.hip -- finite-volume step on the 25-velocity Gauss-Hermite lattice
// (GH5 x GH5, T_ref = 1) for gfx950: van Leer limited upwind fluxes + BGK
// relaxation toward the order-4 Grad-Hermite equilibrium + sensors S_KL,
// S_NEQ, S_PI, S_Q + refinement flags + FP64 sums, in one kernel.
//
// Method (arXiv 2603.13618): explicit Euler FV update eq. finalDiscretePDE,
//   f_i^{n+1} = f_i^n - dt/dx sum_faces v_i f_face + dt/tau (f^eq_i - f_i^n),
// tau = mu/(rho T) (Sec. II.A.2 with p = rho R T, R = 1); the face value is the
// upwind cell value plus half its van Leer slope, 2ab/(a+b) for same-sign
// one-sided differences a, b and 0 otherwise (Sec. II.A.3, last paragraph);
// the equilibrium is the Grad-Hermite expansion to order 4 (Sec. II.A.3),
// which for a 2D Maxwellian factorises into 1D Hermite coefficients
// h_n(u, theta) = E[He_n(X)], X ~ N(u, theta); sensors and sums are taken on
// f^n, the state the collision reads.
//
// Layout and staging: deviations d_i = f_i - w_i rho0 (the constant part
// cancels in every flux difference), population i of cell (x, y) at
// i * pp + y * pr + x (PopLayout: plane-major [25][ny][nx] or row-interleaved
// [ny][25][nx]).  One workgroup per TX x TY tile: each thread keeps its own
// cell's populations in registers, and the stencil neighbours (the tile and
// a two-cell cross-shaped halo) reach LDS one velocity group at a time,
// double-buffered (the double distribution's f kernel stages all 25 f planes
// at once).  Tiles are assigned to workgroups so that the eight XCDs each
// sweep their own band of tile columns row by row: vertically adjacent tiles
// run on the same XCD shortly after one another, so halo rows are served by
// that XCD's L2.
//
// The double distribution (f, g; quasi-equilibrium collision) has its own
// kernel further down: the same fluxes on 50 planes, two passes over the
// velocities (non-equilibrium parts and heat fluxes, then collision and
// fluxes) and five sensors.
#include "lks_device.h"
#include "lks_internal.h"

// FP32 workgroup tile (cells) of the single-distribution kernel and the
// minimum waves per SIMD its register allocation must allow (0 = compiler).
// Measured at 2048^2 (us per step, the current kernel with the non-temporal
// stores): 32 x 4 265.3, 64 x 4 265.2, 32 x 8 268.7, 64 x 2 271.4, 128 x 2
// 289.8; on an earlier build 16 x 8 324.9, 64 x 8 327.6, 32 x 16 339.2 against
// 290.0 for 32 x 8: rows of 16 cells are half a 128-byte line, and the
// staging of 16-wide tiles alone takes as long as the whole step of 32-wide
// ones.
#ifndef LKS_Q25_TX
#define LKS_Q25_TX 32
#endif
#ifndef LKS_Q25_TY
#define LKS_Q25_TY 4
#endif
#ifndef LKS_Q25_WAVES
#define LKS_Q25_WAVES 0
#endif
// FP32 workgroup tile (cells) of the double-distribution kernels and the
// minimum waves per SIMD the f kernel's register allocation must allow (0 =
// compiler's choice).  Left alone the compiler gives the f kernel a budget
// of one wave per SIMD; two waves fit without spilling (three spill).
// Rows of 32 cells are whole 128-byte lines (whole-line reads, and stores
// that may carry the non-temporal hint); four rows keep the workgroup small
// enough for several to share a CU across the barriers.  Step at 2048^2
// (both kernels): 32 x 4 660 us, 32 x 2 685, 32 x 8 683, 64 x 2 690, 64 x 4
// 676, 128 x 2 740, 16 x 8 706, 16 x 16 761; 32 x 4 without the hint 678.
#ifndef LKS_DDF_TX
#define LKS_DDF_TX 32
#endif
#ifndef LKS_DDF_TY
#define LKS_DDF_TY 4
#endif
#ifndef LKS_DDF_WAVES
#define LKS_DDF_WAVES 2
#endif
// FP32 tile of the double distribution's g kernel (its own launch grid):
// rows of 64 cells, two whole 128-byte lines, stage fewer halo columns per
// cell than rows of 32; and the waves per SIMD its register allocation must
// allow (0 = the compiler's choice, four).  Step at 2048^2 (both kernels, the
// f kernel on 32 x 4): g on 64 x 4 637 us, 128 x 4 638, 128 x 2 641, 64 x 8
// 648, 32 x 8 653 (five waves 657), 32 x 4 662, 32 x 16 663, 64 x 2 668;
// five waves on 64 x 4 (89 registers) 641 against 634 on one box.
#ifndef LKS_DDF_G_TX
#define LKS_DDF_G_TX 64
#endif
#ifndef LKS_DDF_G_TY
#define LKS_DDF_G_TY 4
#endif
#ifndef LKS_DDF_G_WAVES
#define LKS_DDF_G_WAVES 0
#endif

namespace lks {

// GH5 nodes (x-node a, y-node b), He_n(xi)/n! and 1D weights, T_ref = 1
__device__ __forceinline__ constexpr double gh5_xi(int a)
{
    return a == 0 ? -2.856970013872805654 : a == 1 ? -1.355626179974265866 : a == 2 ? 0.0
         : a == 3 ? 1.355626179974265866 : 2.856970013872805654;
}
__device__ __forceinline__ constexpr double gh5_w(int a)
{
    return (a == 0 || a == 4) ? 0.011257411327720688933 : (a == 1 || a == 3) ? 0.22207592200561264440
         : 0.53333333333333333333;
}
// He_n(xi_a) / n!, n = 1..4
__device__ __forceinline__ constexpr double gh5_he(int a, int n)
{
    const double s = (a < 2) ? -1.0 : 1.0;
    if (a == 2) return n == 2 ? -0.5 : (n == 4 ? 0.125 : 0.0);
    const bool outer = (a == 0 || a == 4);
    switch (n) {
    case 1: return s * (outer ? 2.856970013872805654 : 1.355626179974265866);
    case 2: return outer ? 3.581138830084189666 : 0.4188611699158103340;
    case 3: return s * (outer ? 2.458078746397754902 : -0.2626023374205813369);
    default: return outer ? 0.8603796100280632220 : -0.1937129433613965553;
    }
}

template <int N, typename F, int I = 0>
__device__ __forceinline__ void sfor25(F&& f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        sfor25<N, F, I + 1>(static_cast<F&&>(f));
    }
}

__device__ __forceinline__ int ghost_index(int j, int n, int bc)
{
    if (bc == 0) {
        j %= n;
        return j < 0 ? j + n : j;
    }
    return j < 0 ? 0 : (j >= n ? n - 1 : j);
}

// Hermite coefficients h_1..h_4 of N(u, 1 + tm1) (h_0 = 1)
template <typename R>
__device__ __forceinline__ void hermite_h(R u, R tm1, R (&h)[5])
{
    const R u2 = u * u;
    h[0] = R(1);
    h[1] = u;
    h[2] = u2 + tm1;
    h[3] = u * (u2 + R(3) * tm1);
    h[4] = u2 * (u2 + R(6) * tm1) + R(3) * tm1 * tm1;
}

// f^eq_i - w_i rho0 for all 25 populations from (rho - rho0, rho, u, theta - 1),
// with the leading "1" of the expansion taken out so nothing cancels:
// f^eq_ab = w_a w_b rho (1 + s_ab), s_ab = Px~_a + Sy~_b[4] + sum_{n=1..3}
// Px_a[n] Sy~_b[4 - n] with Px_a[n] = h_n(u_x) He_n(xi_a)/n! and Px~_a their
// sum over n = 1..4.  Deq25 holds the per-cell factors; group<A>() gives
// the five populations of x-node A, d2q25_deq all 25.  The nodes are
// symmetric, xi_{4-a} = -xi_a, so He_n(xi_{4-a}) = (-1)^n He_n(xi_a): with E
// the even and O the odd powers of the x expansion, s_ab = E + O and
// s_{4-a,b} = E - O, which pair<A>() uses for x-nodes A and 4 - A together
// (d2q25_deq_pairs); Sy~_2 has no odd terms (Sy~_2[1] = 0, Sy~_2[3] =
// Sy~_2[2]).
template <typename R> struct Deq25 {
    R hx[5];
    R sy[5][5];           // Sy~_b[m] = sum_{n=1..m} hy[n] He_n(xi_b)/n!
    R drho, rho;
    __device__ __forceinline__ Deq25(R drho_, R rho_, R ux, R uy, R tm1) : drho(drho_), rho(rho_)
    {
        R hy[5];
        hermite_h(ux, tm1, hx);
        hermite_h(uy, tm1, hy);
#pragma unroll
        for (int b = 0; b < 5; ++b) {
            sy[b][0] = R(0);
#pragma unroll
            for (int m = 1; m < 5; ++m)
                sy[b][m] = (b == 2 && m % 2 == 1) ? sy[b][m - 1] : fma(hy[m], R(gh5_he(b, m)), sy[b][m - 1]);
        }
    }
    // the population loops are unrolled by templates: a pragma gives up when
    // the caller's per-population body is large, and the callers index
    // register arrays by the population
    template <int A, typename F> __device__ __forceinline__ void group(F&& use) const
    {
        R px[5];
        R pt = R(0);
        px[0] = R(1);
#pragma unroll
        for (int n = 1; n < 5; ++n) {
            px[n] = hx[n] * R(gh5_he(A, n));
            pt += px[n];
        }
        sfor25<5>([&](auto bc) {
            constexpr int b = decltype(bc)::value;
            R s = pt + sy[b][4];
#pragma unroll
            for (int n = 1; n < 4; ++n) s += px[n] * sy[b][4 - n];
            use(A, b, R(gh5_w(A) * gh5_w(b)) * (rho * s + drho));
        });
    }
    // x-nodes A and 4 - A (A < 2), population (A, b) before (4 - A, b); the
    // same values as group<A>() and group<4 - A>() up to rounding, in fewer
    // operations
    template <int A, typename F> __device__ __forceinline__ void pair(F&& use) const
    {
        static_assert(A < 2, "pair of x-nodes A and 4 - A");
        R p[5];
#pragma unroll
        for (int n = 1; n < 5; ++n) p[n] = hx[n] * R(gh5_he(A, n));
        const R pe = p[2] + p[4], po = p[1] + p[3];
        sfor25<5>([&](auto bc) {
            constexpr int b = decltype(bc)::value;
            const R e = fma(p[2], sy[b][2], pe + sy[b][4]);
            R o;
            if constexpr (b == 2) o = fma(p[1], sy[b][2], po);
            else o = fma(p[1], sy[b][3], fma(p[3], sy[b][1], po));
            const R w = R(gh5_w(A) * gh5_w(b));             // w_{4-A} = w_A
            use(A, b, w * fma(rho, e + o, drho));
            use(4 - A, b, w * fma(rho, e - o, drho));
        });
    }
};

// all 25 populations in order
template <typename R, typename F>
__device__ __forceinline__ void d2q25_deq(R drho, R rho, R ux, R uy, R tm1, F&& use)
{
    const Deq25<R> e(drho, rho, ux, uy, tm1);
    sfor25<5>([&](auto ac) { e.template group<decltype(ac)::value>(use); });
}

// all 25 populations by mirror pairs of x-nodes: 0 and 4, 1 and 3, then 2
// (population 0 first).  Fewer operations than d2q25_deq, but a caller
// holding many registers across it may need more (the single-distribution
// kernel's rare fallback then cost it a wave per SIMD)
template <typename R, typename F>
__device__ __forceinline__ void d2q25_deq_pairs(R drho, R rho, R ux, R uy, R tm1, F&& use)
{
    const Deq25<R> e(drho, rho, ux, uy, tm1);
    e.template pair<0>(use);
    e.template pair<1>(use);
    e.template group<2>(use);
}

// class of |v|^2 of population (a, b) on GH5 x GH5: 0 centre, 1 one inner
// abscissa, 2 one outer, 3 two inner, 4 inner and outer, 5 two outer
__device__ __forceinline__ constexpr int v2_class(int a, int b)
{
    const int p = a == 2 ? 0 : (a == 1 || a == 3) ? 1 : 2;
    const int q = b == 2 ? 0 : (b == 1 || b == 3) ? 1 : 2;
    return p == 0 ? q : q == 0 ? p : p + q + 1;
}

// pairwise (tree) sum of a register array: rounding error O(log N) instead
// of O(N) terms deep
template <typename R, int N>
__device__ __forceinline__ R pairwise_sum(R (&v)[N])
{
#pragma unroll
    for (int len = N; len > 1; len = (len + 1) / 2) {
#pragma unroll
        for (int k = 0; k < len / 2; ++k) v[k] = v[2 * k] + v[2 * k + 1];
        if (len % 2) v[len / 2] = v[len - 1];
    }
    return v[0];
}

// half van Leer slope ab/(a+b) for same-sign a, b, else 0
template <typename R>
__device__ __forceinline__ R vl_half(R a, R b)
{
    const R p = a * b;
    return p > R(0) ? p * rcp(a + b) : R(0);
}
// FP32: max(ab, 0) times 1/(a+b) with the legacy multiply, whose zero times
// anything (the infinite reciprocal of a + b = 0 included) is +0: the same
// value as the select above (a, b of one sign give a + b != 0 and the same
// product), one VALU instruction fewer than compare and select (2048^2
// single distribution: 276.5 against 280.0 us per step).  Called as the
// compiler's intrinsic, not as inline assembly, so that the compiler still
// inserts the wait state gfx950 needs between the reciprocal and a VALU
// instruction that reads it (inline assembly reading the reciprocal at once
// got stale values).  LKS_VL_LEGACY 0 builds the select form.
#ifndef LKS_VL_LEGACY
#define LKS_VL_LEGACY 1
#endif
#if LKS_VL_LEGACY
extern "C" __device__ float lks_fmul_legacy(float, float) __asm("llvm.amdgcn.fmul.legacy");
template <>
__device__ __forceinline__ float vl_half<float>(float a, float b)
{
    return lks_fmul_legacy(fmaxf(a * b, 0.0f), rcp(a + b));
}
#endif

// Population stores of the D2Q25 kernels, with the non-temporal hint (NTS)
// when the two state buffers exceed the last-level cache: the next step's
// loads come from HBM either way, and the hint keeps the written lines from
// evicting the rows and halo lines other tiles are still to read (2048^2
// single distribution: read traffic 612 -> 450 MB per step, 276.3 -> 269.6
// us)
template <bool NT, typename T>
__device__ __forceinline__ void put_pop(T* p, T v)
{
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// f_face(j + 1/2) - f_face(j - 1/2) for the stencil q[-2..2] (q[2] = cell j),
// upwind for velocity sign SIGN: the difference of the two upwind cells plus
// the difference of their limited half slopes
template <typename R, int SIGN>
__device__ __forceinline__ R flux_diff(R qm2, R qm1, R q0, R qp1, R qp2)
{
    const R dl = q0 - qm1, dr = qp1 - q0;
    if constexpr (SIGN > 0)
        return dl + (vl_half(dl, dr) - vl_half(qm1 - qm2, dl));
    else
        return dr - (vl_half(dr, qp2 - qp1) - vl_half(dl, dr));
}

// -(dt/dx) xi_a for the five abscissae, each rounded once from FP64, so the
// advection of a population is one multiply-add per direction
template <typename R> struct AdvScale {
    R s3, s4;   // (dt/dx) xi_3, (dt/dx) xi_4; xi_1 = -xi_3, xi_0 = -xi_4, xi_2 = 0
    __device__ __forceinline__ explicit AdvScale(const D2Q25Args& a)
        : s3(R(a.dt / a.dx * gh5_xi(3))), s4(R(a.dt / a.dx * gh5_xi(4))) {}
    __device__ __forceinline__ R neg(int i) const { return i == 3 ? -s3 : i == 4 ? -s4 : i == 1 ? s3 : s4; }
};

// q . v of population (ia, ib), without the terms of a zero component
template <typename R>
__device__ __forceinline__ R q_dot_v(R qx, R qy, int ia, int ib)
{
    if (ia == 2) return qy * R(gh5_xi(ib));
    if (ib == 2) return qx * R(gh5_xi(ia));
    return fma(qx, R(gh5_xi(ia)), qy * R(gh5_xi(ib)));
}

// One population's extension sums: ExtAcc::add, and the entropy-flux sums
// of the dissipations, V += c v ln(h/w) and W += c v ln(h/h^eq) with ln(h/w)
// = ln(h^eq/w) + ln(1 + x).  lt is ln(h^eq/w): taken here from t = h^eq/w - 1
// unless lt_given, and returned.  Each logarithm is taken once, inside the
// branch of the mask bits that need it (V needs both sums of the kind of L
// and S, W those of S).
template <typename R>
__device__ __forceinline__ void ext_add_vw(ExtAcc<R>& e, const ExtNeed& need, bool needV, bool needW, R fneq_,
                                           R x_, R f_, R t_, bool lt_given, R& lt, R cvx, R cvy, R& vx, R& vy,
                                           R& wx, R& wy)
{
    const R fneq = pin(fneq_), x = pin(x_), f = pin(f_);
    e.kn += fabs(x);
    if (need.L) {
        if (!lt_given) lt = ln1p_fast(pin(t_));
        e.L += fneq * lt;
    }
    if (need.S) {
        const R lx = ln1p_fast(x);
        e.shkl += fneq * lx;
        if (needV) {
            const R l = lt + lx;
            vx += cvx * l;
            vy += cvy * l;
        }
        if (needW) {
            wx += cvx * lx;
            wy += cvy * lx;
        }
    }
    if (need.A) {
        const R y = fneq * rcp(f);             // f^neq / f
        const R t1 = fneq * y, t2 = t1 * y, t3 = t2 * y;
        e.a1 += t1;
        e.a2 += t2;
        e.a3 += t3;
        e.a4 += t3 * y;
    }
}

// o - (dt/dx) (xi_ia dF_x + xi_ib dF_y): the flux divergence of population
// (ia, ib), value d, whose staged plane is t, added to o
template <typename R>
__device__ __forceinline__ R advect(R o, const AdvScale<R>& sc, const R* t, const int (&rb)[5], int tx, R d,
                                    int ia, int ib)
{
    if (ia != 2) {
        const R* row = t + rb[2] + tx;
        o = fma(sc.neg(ia), ia > 2 ? flux_diff<R, 1>(row[-2], row[-1], d, row[1], R(0))
                                   : flux_diff<R, -1>(R(0), row[-1], d, row[1], row[2]), o);
    }
    if (ib != 2)
        o = fma(sc.neg(ib), ib > 2 ? flux_diff<R, 1>(t[rb[0] + tx], t[rb[1] + tx], d, t[rb[3] + tx], R(0))
                                   : flux_diff<R, -1>(R(0), t[rb[1] + tx], d, t[rb[3] + tx], t[rb[4] + tx]), o);
    return o;
}

// Workgroup -> tile.  Consecutive workgroup ids go to the eight XCDs in turn
// (id mod 8), each with its own L2, so the order decides which halo rows and
// columns a tile finds in its XCD's L2.  LKS_Q25_XCD_MAP 1 (default): XCD k
// sweeps row band k of the tile rows row by row, so the halo columns always
// come from its own L2 and only the band's first and last tile rows read
// halo rows another XCD loaded; 0: XCD k sweeps column band k of the tile
// columns row by row (every band edge reads its halo columns from another
// XCD's band); 2: plain row-major order.  Measured at 2048^2 (FP32 kernel
// time per step, a 3-wave build of the single-distribution kernel): single
// distribution 354 / 376 / 362 us for maps 1 / 0 / 2, double distribution
// 799 / 808 / 877 us.  Bands swept column by column were worse (read bytes
// per step 913 and 1422 MB against 614 MB, 282 and 329 us against 277 us):
// the x-halo of a 32-wide tile is two floats of each neighbour's 128-byte
// rows, so horizontal neighbours must run close together in time.  Shapes
// that do not divide into 8 bands use row-major order.
#ifndef LKS_Q25_XCD_MAP
#define LKS_Q25_XCD_MAP 1
#endif
__device__ __forceinline__ void xcd_tile(const D2Q25Args& a, int& tile_x, int& tile_y)
{
    const int b = blockIdx.x;
    if (LKS_Q25_XCD_MAP == 0 && a.tiles_x % 8 == 0) {
        const int bw = a.tiles_x / 8, l = b / 8;
        tile_x = (b % 8) * bw + l % bw;
        tile_y = l / bw;
    } else if (LKS_Q25_XCD_MAP == 1 && a.tiles_y % 8 == 0) {
        const int bh = a.tiles_y / 8, l = b / 8;
        tile_x = l % a.tiles_x;
        tile_y = (b % 8) * bh + l / a.tiles_x;
    } else {
        tile_x = b % a.tiles_x;
        tile_y = b / a.tiles_x;
    }
}

template <int TX, int TY> struct Tile {
    static constexpr int kPlane = 4 * TX + TY * (TX + 4);
    // LDS offset of row r (-2 .. TY+1) at column 0 (columns -2..TX+1 on
    // interior rows, 0..TX-1 on halo rows)
    __device__ static int rowbase(int r)
    {
        return r < 0 ? (r + 2) * TX : (r < TY ? 2 * TX + r * (TX + 4) + 2 : 2 * TX + TY * (TX + 4) + (r - TY) * TX);
    }
};

// The loads that stage a TX x TY tile and its two-cell cross halo: each
// thread's own cell, up to HR halo-row cells and one halo-column cell, at
// the same offsets in every population plane.  Groups of NG planes go
// through LDS one at a time: load() puts a group's halo values in registers
// (in flight while the previous group is computed), write() stores them and
// the threads' own values into one LDS buffer.  Planes are kStride floats
// apart in LDS, the last one a spare slot: a thread without a halo cell
// loads its own cell again and writes it there, so no load or store is
// conditional (a branch around a load makes the compiler wait for every
// load in flight where the branches join, the prefetched group's included).
template <typename S, int TX, int TY> struct TileStage {
    using R = typename Store<S>::real;
    using raw = typename Store<S>::raw;
    using T = Tile<TX, TY>;
    static constexpr int NT = TX * TY;
    static constexpr int HR = (4 * TX + NT - 1) / NT;
    static constexpr int kStride = T::kPlane + 1;
    long long own, hoff[HR], coff;
    int hlds[HR], clds, olds;

    __device__ __forceinline__ TileStage(const D2Q25Args& a, int X0, int Y0, int tx, int ty)
    {
        const int nx = a.nx, ny = a.ny;
        own = (long long)ghost_index(Y0 + ty, ny, a.bc_y) * a.L.pr + ghost_index(X0 + tx, nx, a.bc_x);
#pragma unroll
        for (int k = 0; k < HR; ++k) {
            const int h = threadIdx.x + k * NT;
            const int hr = h / TX, c = h % TX;
            const int r = hr < 2 ? hr - 2 : TY + hr - 2;
            const bool halo = h < 4 * TX;
            hoff[k] = halo ? (long long)ghost_index(Y0 + r, ny, a.bc_y) * a.L.pr + ghost_index(X0 + c, nx, a.bc_x)
                           : own;
            hlds[k] = halo ? T::rowbase(r) + c : T::kPlane;
        }
        coff = own;
        clds = T::kPlane;
        if (threadIdx.x < 4 * TY) {
            const int hc = threadIdx.x % 4, r = threadIdx.x / 4;
            const int c = hc < 2 ? hc - 2 : TX + hc - 2;
            coff = (long long)ghost_index(Y0 + r, ny, a.bc_y) * a.L.pr + ghost_index(X0 + c, nx, a.bc_x);
            clds = T::rowbase(r) + c;
        }
        olds = T::rowbase(ty) + tx;
    }
    // halo values of planes p0 .. p0 + NG - 1
    template <int NG>
    __device__ __forceinline__ void load(const raw* __restrict__ fin, long long pp, int p0, R (&vh)[NG][HR],
                                         R (&vc)[NG]) const
    {
        sfor25<NG>([&](auto pc) {
            constexpr int p = decltype(pc)::value;
            const raw* src = fin + (p0 + p) * pp;
#pragma unroll
            for (int k = 0; k < HR; ++k) vh[p][k] = Store<S>::to_real(src[hoff[k]]);
            vc[p] = Store<S>::to_real(src[coff]);
        });
    }
    // a group into buf (NG planes kStride apart): own values mine[Q0 ..], halo vh, vc
    template <int NG, int Q0, int NQ>
    __device__ __forceinline__ void write(R* buf, const R (&mine)[NQ], const R (&vh)[NG][HR], const R (&vc)[NG]) const
    {
        sfor25<NG>([&](auto pc) {
            constexpr int p = decltype(pc)::value;
            R* dst = buf + p * kStride;
            dst[olds] = mine[Q0 + p];
#pragma unroll
            for (int k = 0; k < HR; ++k) dst[hlds[k]] = vh[p][k];
            dst[clds] = vc[p];
        });
    }
};

template <int NW>
__device__ __forceinline__ void block_sums_n(double (&acc)[kNsums], double* __restrict__ out)
{
    __shared__ double red[NW][kNsums];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
#pragma unroll
    for (int k = 0; k < kNsums; ++k) acc[k] = wave_sum(acc[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < kNsums; ++k) red[wave][k] = acc[k];
    }
    __syncthreads();
    if (threadIdx.x < kNsums) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) s += red[w][threadIdx.x];
        out[threadIdx.x] = s;
    }
}

template <typename S> struct Q25Waves { static constexpr int v = 1; };
template <> struct Q25Waves<float> { static constexpr int v = LKS_Q25_WAVES > 0 ? LKS_Q25_WAVES : 1; };

// One workgroup per TX x TY tile.  Every thread keeps its own cell's 25
// values in registers (the moments need all of them first); the stencil
// neighbours reach LDS one velocity group at a time (the five populations of
// one x-node: the tile and its two-cell cross halo), double-buffered, so the
// halo loads of group a + 1 are in flight while group a is computed.  Wide
// tiles keep every row piece of a load a whole number of 128-byte lines.
// Unlike TileStage, only the threads with a halo cell load one: here that
// keeps the kernel at 121 registers (four waves per SIMD) and measured 7 %
// faster than the unconditional form.
template <typename S, int TX, int TY, bool EXT = false, bool EDGE = true, bool NTS = false>
__global__ __launch_bounds__(TX * TY) __attribute__((amdgpu_waves_per_eu(Q25Waves<S>::v))) void d2q25_kernel(D2Q25Args a, const typename Store<S>::raw* __restrict__ fin,
                                                   typename Store<S>::raw* __restrict__ fout,
                                                   typename Store<S>::real* __restrict__ sens,
                                                   uint8_t* __restrict__ flags,
                                                   double* __restrict__ partials,
                                                   unsigned long long* __restrict__ faults)
{
    using R = typename Store<S>::real;
    using T = Tile<TX, TY>;
    constexpr int NT = TX * TY;
    constexpr int NG = 5;                      // planes per staged group
    __shared__ R lds[2][NG * T::kPlane];

    const int nx = a.nx, ny = a.ny;
    const long long plane = a.plane;
    int tile_x, tile_y;
    xcd_tile(a, tile_x, tile_y);
    const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
    const int X0 = tile_x * TX, Y0 = tile_y * TY;
    const int X = X0 + tx, Y = Y0 + ty;
    // EDGE = false: the grid is a whole number of tiles, every thread owns a
    // cell, and no store needs a branch around it (a branch per store cuts
    // the arithmetic of a velocity group into separate scheduling regions)
    const bool active = !EDGE || (X < nx && Y < ny);
    const int gxc = ghost_index(X, nx, a.bc_x), gyc = ghost_index(Y, ny, a.bc_y);
    constexpr int HR = (4 * TX + NT - 1) / NT;
    const long long own = (long long)gyc * a.L.pr + gxc;
    long long hoff[HR];
    int hlds[HR];
#pragma unroll
    for (int k = 0; k < HR; ++k) {
        const int h = threadIdx.x + k * NT;
        const int hr = h / TX, c = h % TX;
        const int r = hr < 2 ? hr - 2 : TY + hr - 2;
        hoff[k] = (long long)ghost_index(Y0 + r, ny, a.bc_y) * a.L.pr + ghost_index(X0 + c, nx, a.bc_x);
        hlds[k] = h < 4 * TX ? T::rowbase(r) + c : -1;
    }
    long long coff = 0;
    int clds = -1;
    if (threadIdx.x < 4 * TY) {
        const int hc = threadIdx.x % 4, r = threadIdx.x / 4;
        const int c = hc < 2 ? hc - 2 : TX + hc - 2;
        coff = (long long)ghost_index(Y0 + r, ny, a.bc_y) * a.L.pr + ghost_index(X0 + c, nx, a.bc_x);
        clds = T::rowbase(r) + c;
    }
    const int olds = T::rowbase(ty) + tx;

    // ---- own-cell values of all 25 planes, and the halo of group 0
    R vin[25];
    sfor25<25>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        vin[i] = Store<S>::to_real(fin[i * a.L.pp + own]);
    });
    R vh[NG][HR], vc[NG];
    auto load_group = [&](auto gc) {
        constexpr int g = decltype(gc)::value;
        sfor25<NG>([&](auto pc) {
            constexpr int p = decltype(pc)::value;
            const typename Store<S>::raw* src = fin + (NG * g + p) * a.L.pp;
#pragma unroll
            for (int k = 0; k < HR; ++k) vh[p][k] = hlds[k] >= 0 ? Store<S>::to_real(src[hoff[k]]) : R(0);
            vc[p] = clds >= 0 ? Store<S>::to_real(src[coff]) : R(0);
        });
    };
    auto write_group = [&](auto gc) {
        constexpr int g = decltype(gc)::value;
        R* buf = lds[g & 1];
        sfor25<NG>([&](auto pc) {
            constexpr int p = decltype(pc)::value;
            R* dst = buf + p * T::kPlane;
            dst[olds] = vin[NG * g + p];
#pragma unroll
            for (int k = 0; k < HR; ++k)
                if (hlds[k] >= 0) dst[hlds[k]] = vh[p][k];
            if (clds >= 0) dst[clds] = vc[p];
        });
    };
    load_group(std::integral_constant<int, 0>{});

    // ---- moments and cell state: rho, u, theta - 1, relaxation factor
    const R rho0 = R(a.rho0);
    R drho = R(0), jx = R(0), jy = R(0), edev = R(0);
    sfor25<25>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        constexpr int ia = i / 5, ib = i % 5;
        const R v = vin[i];
        drho += v;
        if (ia != 2) jx += R(gh5_xi(ia)) * v;
        if (ib != 2) jy += R(gh5_xi(ib)) * v;
        edev += R(0.5 * (gh5_xi(ia) * gh5_xi(ia) + gh5_xi(ib) * gh5_xi(ib))) * v;
    });
    const R rho = rho0 + drho;
    const R irho = rcp(rho);
    const R ux = jx * irho, uy = jy * irho;
    // T = (2E/rho - |u|^2)/2 with E = rho0 + edev (sum_i w_i |v_i|^2/2 = 1)
    const R tm1 = (edev - drho) * irho - R(0.5) * (ux * ux + uy * uy);
    const AdvScale<R> adv(a);
    const R B = R(a.dt / a.mu) * rho * (R(1) + tm1);   // dt / tau
    const Deq25<R> eq(drho, rho, ux, uy, tm1);

    write_group(std::integral_constant<int, 0>{});
    __syncthreads();

    const int rb[5] = {T::rowbase(ty - 2), T::rowbase(ty - 1), T::rowbase(ty), T::rowbase(ty + 1),
                       T::rowbase(ty + 2)};
    // pxx, pxy: the non-equilibrium stress behind S_PI (below)
    R kl = R(0), neq = R(0), qx = R(0), qy = R(0), pxx = R(0), pxy = R(0);
    R xmin = R(0), xmax = R(0), feqmin = R(0);
    bool first = true;
    const long long off = (long long)Y * nx + X;
    const long long poff = a.L.at(0, Y, X);
    sfor25<5>([&](auto gc) {
        constexpr int g = decltype(gc)::value;
        // the next group's halo is in flight while this one is computed
        if constexpr (g + 1 < 5) load_group(std::integral_constant<int, g + 1>{});
        const R* buf = lds[g & 1];
        eq.template group<g>([&](int ia, int ib, R deq) {
            const int i = 5 * ia + ib;
            const R* t = buf + ib * T::kPlane;
            const R d = vin[i];
            const R fneq = d - deq;
            const R feq = R(gh5_w(ia) * gh5_w(ib)) * rho0 + deq;
            const R x = fneq * rcp(feq);
            kl += (fneq * x) * kl_series_short(x);     // series branch; fallback below
            xmax = first ? fabs(x) : fmax(xmax, fabs(x));
            feqmin = first ? feq : fmin(feqmin, feq);
            first = false;
            neq += fabs(fneq);
            // explicit multiply-adds (contraction fixed in every instantiation)
            if (ia != ib && ia != 4 - ib)
                pxx = fma(R(0.5 * (gh5_xi(ia) * gh5_xi(ia) - gh5_xi(ib) * gh5_xi(ib))), fneq, pxx);
            if (ia != 2 && ib != 2) pxy = fma(R(gh5_xi(ia) * gh5_xi(ib)), fneq, pxy);
            const R vx = R(gh5_xi(ia)), vy = R(gh5_xi(ib));
            const R e = R(0.5) * (vx * vx + vy * vy);
            qx += vx * e * fneq;
            qy += vy * e * fneq;
            // collision, then the flux divergence (dimension by dimension,
            // upwind + van Leer)
            const R o = advect<R>(fma(B, deq - d, d), adv, t, rb, tx, d, ia, ib);
            if (active) put_pop<NTS>(fout + i * a.L.pp + poff, Store<S>::from_real(o));
        });
        if constexpr (g + 1 < 5) {
            write_group(std::integral_constant<int, g + 1>{});
            __syncthreads();
        }
    });
    // rare: some population far from equilibrium (or NaN): the longer series
    // or the closed form, population by population, and the smallest x
    // (x > -1 is f > 0; on the short-series branch |x| <= 0.03 implies it)
    const bool far = !(xmax <= KlShortCut<R>::v);
    if (far) {
        kl = R(0);
        first = true;
        d2q25_deq<R>(drho, rho, ux, uy, tm1, [&](int ia, int ib, R deq) {
            const R d = vin[5 * ia + ib];
            const R feq = R(gh5_w(ia) * gh5_w(ib)) * rho0 + deq;
            const R x = (d - deq) * rcp(feq);
            xmin = first ? x : fmin(xmin, x);
            first = false;
            kl += feq * kl_phi(x);
        });
    }

    // Non-equilibrium stress P = sum v v f^neq.  T comes from this cell's own
    // energy and the order-4 equilibrium carries the Maxwellian's energy
    // exactly (GH5 integrates degree 9), so tr P = 2 (E - E^eq) = 0 and P =
    // [[pxx, pxy], [pxy, -pxx]] with pxx = sum (xi_a^2 - xi_b^2)/2 f^neq: the
    // trace, where the rounding of the 25 equilibrium populations
    // concentrates, never enters (FP32 error about 6x smaller than the three
    // components summed separately, and 20 fewer multiply-adds).
    const R pyy = -pxx;
    const bool fault = !(feqmin > R(0)) || (far && !(xmin > R(-1))) || !(kl == kl);
    const R s_kl = fault ? R(INFINITY) : kl;
    // explicit multiply-adds: the same bits in every instantiation
    const R s_pi = sqrt_r(R(2) * fma(pxx, pxx, pxy * pxy));
    const R s_q = sqrt_r(fma(qx, qx, qy * qy));
    double acc[kNsums];
#pragma unroll
    for (int k = 0; k < kNsums; ++k) acc[k] = 0.0;
    if (active) {
        const R sv[4] = {s_kl, neq, s_pi, s_q};
        LevelAcc lv;
#pragma unroll
        for (int s = 0; s < 4; ++s) lv.add(sv[s], R(a.thr[s][0]), R(a.thr[s][1]));
        if constexpr (EXT) {
            // A separate pass on opaque copies (pin) of the moments and of the
            // cell's populations, after the base arithmetic: no base
            // expression gains a use, so the base results do not depend on
            // the extension.
            const R drho_p = pin(drho), rho_p = pin(rho), ux_p = pin(ux), uy_p = pin(uy),
                    tm1_p = pin(tm1), rho0_p = pin(rho0);
            ExtAcc<R> xa;
            const ExtNeed need(a.x.mask);
            d2q25_deq<R>(drho_p, rho_p, ux_p, uy_p, tm1_p, [&](int ia, int ib, R deq) {
                const R d = pin(vin[5 * ia + ib]);
                const R w = R(gh5_w(ia) * gh5_w(ib));
                const R fneq = d - deq;
                const R x = fneq * rcp(w * rho0_p + deq);
                // f = w rho0 + d; f^eq/w - 1 = (rho0 - 1) + deq/w
                xa.add(need, fneq, x, w * rho0_p + d,
                       (rho0_p - R(1)) + deq * R(1.0 / (gh5_w(ia) * gh5_w(ib))));
            });
            // tau = mu/(rho T), the configured mu
            R xv[kNumExt];
            const R inv_mu = R(1.0 / a.mu);
            ext_finish<R>(xa, pin(kl), fault, rho_p * (R(1) + tm1_p) * inv_mu, inv_mu, pxx, pxy, pyy,
                          ux_p, uy_p, pin(qx), pin(qy), true, xv);
#pragma unroll
            for (int q = 0; q < kNumExt; ++q) {
                if (a.x.plane[q] >= 0) sens[a.x.plane[q] * plane + off] = xv[q];
                if (a.mask & (1u << (kExtFlagShift + q))) lv.add(xv[q], R(a.x.thr[q][0]), R(a.x.thr[q][1]));
            }
        }
        sens[off] = s_kl;
        sens[plane + off] = neq;
        sens[2 * plane + off] = s_pi;
        sens[3 * plane + off] = s_q;
        flags[off] = fault ? uint8_t(0x82) : uint8_t(lv.level());
        if (fault) atomicAdd(faults, 1ull);
        acc[0] = (double)drho;
        acc[1] = (double)jx;
        acc[2] = (double)jy;
        acc[3] = (double)edev;
        acc[4] = (double)s_kl;
        acc[5] = (double)neq;
        acc[6] = (double)s_pi;
        acc[7] = (double)s_q;
    }
    block_sums_n<NT / kWave>(acc, partials + (long long)blockIdx.x * kNsums);
}

// ---------------------------------------------------------------------------
// Double distribution (f, g) on the 25-velocity lattice with the
// quasi-equilibrium collision (Sec. II.A.1-3, eqs. new_collision_fi,
// finalDiscretePDE): f carries mass, momentum and translational energy, g the
// non-translational internal energy, g^eq = (C_v - D/2) T f^eq (eq.
// energy_eq_1_rykov), E = sum (g + |v|^2/2 f) = rho (C_v T + |u|^2/2).  With
// the heat flux quasi-conserved (Pr <= 1): f* = f^eq + w (q_f . v)(|v|^2/4 - 1)
// (Grad heat-flux term of the translational heat flux q_f of f), g* = g^eq +
// w (q_g . v) (q_g = sum (v - u) g), Omega = -(f - f*)/tau1 - (f* - f^eq)/tau2,
// tau1 = mu/(rho T), tau2 = tau1/Pr.  Both distributions take the same van
// Leer fluxes.  Sensors: |sum f ln(f/f^eq)| + |sum g ln(g/g^eq)|, sum |f^neq| +
// sum |g^neq|, S_PI of f, |sum v g^neq + sum v |v|^2/2 f^neq|, and the QE
// sensor sum |f* - f^eq| + sum |g* - g^eq| (eqs. HKL-sensor, sensor-neq-kin,
// sensor-TauNS-kin, sensor-qNSF-kin-ryk, Sensor-qe-kin).
// Storage: 50 populations per cell, f deviations from w rho0, then g
// deviations from (C_v - 1) w rho0.
//
// The step is two kernels.  d2q25_ddf_kernel stages f (25 planes, the tile
// and its two-cell cross halo) in LDS and keeps the own-cell g values in
// registers (the moments need them).  Pass 1 over the velocities takes the
// non-equilibrium parts of both: the sensors and the heat fluxes q_f = 1/2
// sum |c|^2 c f^neq, q_g = sum c g^neq (c = v - u; the equilibria carry none,
// so no cancellation), and keeps the 25 equilibrium deviations for pass 2,
// which applies the collision and the fluxes to f and hands drho, u, T - 1
// and q_g of each cell to d2q25_ddf_g_kernel, which updates g.
// ---------------------------------------------------------------------------
// the register hint applies to FP32 storage only (FP64 values take two
// registers each: there the hint would spill hundreds)
template <typename S> struct DdfWaves { static constexpr int v = 1; };
template <> struct DdfWaves<float> { static constexpr int v = LKS_DDF_WAVES > 0 ? LKS_DDF_WAVES : 1; };
template <typename S> struct DdfGWaves { static constexpr int v = 1; };
template <> struct DdfGWaves<float> { static constexpr int v = LKS_DDF_G_WAVES > 0 ? LKS_DDF_G_WAVES : 1; };

template <typename S, int TX, int TY, bool EXT = false, bool EDGE = true, bool NTS = false>
__global__ __launch_bounds__(TX * TY) __attribute__((amdgpu_waves_per_eu(DdfWaves<S>::v))) void d2q25_ddf_kernel(
    D2Q25Args a, const typename Store<S>::raw* __restrict__ fin, typename Store<S>::raw* __restrict__ fout,
    typename Store<S>::real* __restrict__ sens, uint8_t* __restrict__ flags, double* __restrict__ partials,
    unsigned long long* __restrict__ faults)
{
    using R = typename Store<S>::real;
    using T = Tile<TX, TY>;
    constexpr int NT = TX * TY;
    __shared__ R lds[25 * T::kPlane];

    const int nx = a.nx, ny = a.ny;
    const long long plane = a.plane;
    int tile_x, tile_y;
    xcd_tile(a, tile_x, tile_y);
    const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
    const int X0 = tile_x * TX, Y0 = tile_y * TY;
    const int X = X0 + tx, Y = Y0 + ty;
    const bool active = !EDGE || (X < nx && Y < ny);     // EDGE: as in d2q25_kernel
    const int gxc = ghost_index(X, nx, a.bc_x), gyc = ghost_index(Y, ny, a.bc_y);

    constexpr int HR = (4 * TX + NT - 1) / NT;
    const long long own = (long long)gyc * a.L.pr + gxc;
    long long hoff[HR];
    int hlds[HR];
#pragma unroll
    for (int k = 0; k < HR; ++k) {
        const int h = threadIdx.x + k * NT;
        const int hr = h / TX, c = h % TX;
        const int r = hr < 2 ? hr - 2 : TY + hr - 2;
        hoff[k] = (long long)ghost_index(Y0 + r, ny, a.bc_y) * a.L.pr + ghost_index(X0 + c, nx, a.bc_x);
        hlds[k] = h < 4 * TX ? T::rowbase(r) + c : -1;
    }
    long long coff = 0;
    int clds = -1;
    if (threadIdx.x < 4 * TY) {
        const int hc = threadIdx.x % 4, r = threadIdx.x / 4;
        const int c = hc < 2 ? hc - 2 : TX + hc - 2;
        coff = (long long)ghost_index(Y0 + r, ny, a.bc_y) * a.L.pr + ghost_index(X0 + c, nx, a.bc_x);
        clds = T::rowbase(r) + c;
    }
    const int olds = T::rowbase(ty) + tx;
    const int rb[5] = {T::rowbase(ty - 2), T::rowbase(ty - 1), T::rowbase(ty), T::rowbase(ty + 1),
                       T::rowbase(ty + 2)};

    // stage planes [p0, p0 + 25) with their halo; own-cell values into own_v
    // (loaded here unless own_loaded)
    auto stage = [&](int p0, R (&own_v)[25], bool own_loaded) {
        R vh[HR][25], vc[25];
        sfor25<25>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            const typename Store<S>::raw* src = fin + (p0 + i) * a.L.pp;
            if (!own_loaded) own_v[i] = Store<S>::to_real(src[own]);
#pragma unroll
            for (int k = 0; k < HR; ++k) vh[k][i] = hlds[k] >= 0 ? Store<S>::to_real(src[hoff[k]]) : R(0);
            vc[i] = clds >= 0 ? Store<S>::to_real(src[coff]) : R(0);
        });
        sfor25<25>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            R* dst = lds + i * T::kPlane;
            dst[olds] = own_v[i];
#pragma unroll
            for (int k = 0; k < HR; ++k)
                if (hlds[k] >= 0) dst[hlds[k]] = vh[k][i];
            if (clds >= 0) dst[clds] = vc[i];
        });
    };

    // ---- own-cell g values, then f staged with its halo
    R fc[25], gc[25];
    sfor25<25>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        gc[i] = Store<S>::to_real(fin[(25 + i) * a.L.pp + own]);
    });
    stage(0, fc, false);

    // ---- moments: sum d, sum v d, sum |v|^2 d of f and sum dg of g
    const R rho0 = R(a.rho0);
    const R cv = R(a.cv);
    // The energy moments m2 = sum |v|^2 d and dg0 = sum dg are summed with
    // short rounding chains: m2 over the five classes of |v|^2 (four or eight
    // populations each), dg0 pairwise.  S_KL's largest term, sum g^neq below,
    // is a small difference of them (single-step FP32 error of S_KL on the
    // 128^2 Riemann quadrants: 1.2e-5 with plain running sums, about 6e-6
    // this way in a float emulation)
    R drho = R(0), jx = R(0), jy = R(0);
    R sc[6] = {R(0), R(0), R(0), R(0), R(0), R(0)}, eg[25];
    sfor25<25>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        constexpr int ia = i / 5, ib = i % 5;
        const R v = fc[i];
        drho += v;
        if (ia != 2) jx += R(gh5_xi(ia)) * v;
        if (ib != 2) jy += R(gh5_xi(ib)) * v;
        sc[v2_class(ia, ib)] += v;
        eg[i] = gc[i];
    });
    constexpr double x3 = gh5_xi(3) * gh5_xi(3), x4 = gh5_xi(4) * gh5_xi(4);
    const R m2 = fma(R(2 * x4), sc[5], fma(R(x3 + x4), sc[4], fma(R(2 * x3), sc[3], fma(R(x4), sc[2], R(x3) * sc[1]))));
    const R dg0 = pairwise_sum(eg);
    const R rho = rho0 + drho;
    const R irho = rcp(rho);
    const R ux = jx * irho, uy = jy * irho;
    // C_v (T - 1) = (E - C_v rho)/rho - |u|^2/2 with E - C_v rho = dg0 + m2/2
    // - C_v drho (sum_i w_i = 1, sum_i w_i |v_i|^2/2 = 1: the reference parts cancel)
    const R tm1 = ((dg0 + R(0.5) * m2 - cv * drho) * irho - R(0.5) * (ux * ux + uy * uy)) * R(1.0 / a.cv);
    const R Tc = R(1) + tm1;
    const R gfac = cv - R(1);                              // g^eq = (C_v - 1) T f^eq

    // ---- pass 1: non-equilibrium parts of f and g (sensors, heat fluxes)
    // sum g^neq = sum g - (C_v - 1) T rho, with T from the total energy:
    // (dg0 - (C_v - 1)(m2/2 - rho |u|^2/2)) / C_v, the same value as summing
    // the 25 g^neq_i, without the rounding of the equilibrium terms
    const R gsum = fma(-gfac, fma(R(0.5), m2, -(R(0.5) * rho) * fma(ux, ux, uy * uy)), dg0) * R(1.0 / a.cv);
    R klf = R(0), klg = R(0), neq = R(0), pxx = R(0), pxy = R(0), pyy = R(0), qfx = R(0), qfy = R(0),
      qgx = R(0), qgy = R(0);
    // the reach of the KL series (the largest |x|, |y|) and positivity (the
    // smallest f^eq, and the smallest x, y: x > -1 is f > 0).  g^eq = (C_v - 1)
    // T f^eq, so g^eq > 0 wherever f^eq > 0 and T > 0, and 1/g^eq is 1/f^eq
    // times igT = 1/((C_v - 1) T)
    R xmax = R(0), xlo = R(0), eqmin = R(0);
    const R igT = rcp(gfac * Tc);
    R deqv[25];
    d2q25_deq_pairs<R>(drho, rho, ux, uy, tm1, [&](int ia, int ib, R deq) {
        const int i = 5 * ia + ib;
        const R w = R(gh5_w(ia) * gh5_w(ib));
        const R vx = R(gh5_xi(ia)), vy = R(gh5_xi(ib));
        deqv[i] = deq;
        const R fneq = fc[i] - deq;
        const R feq = w * rho0 + deq;
        const R rf = rcp(feq);
        const R x = fneq * rf;
        // deviation of g^eq from (C_v - 1) w rho0: (C_v - 1)(T deq + (T - 1) w rho0)
        const R dgeq = gfac * (Tc * deq + tm1 * (w * rho0));
        const R gneq = gc[i] - dgeq;
        const R y = gneq * (rf * igT);
        klf += (fneq * x) * kl_series_short(x);
        klg += (gneq * y) * kl_series_short(y);
        xmax = i == 0 ? fmax(fabs(x), fabs(y)) : fmax(xmax, fmax(fabs(x), fabs(y)));
        xlo = i == 0 ? fmin(x, y) : fmin(xlo, fmin(x, y));
        eqmin = i == 0 ? feq : fmin(eqmin, feq);
        neq += fabs(fneq) + fabs(gneq);
        // explicit multiply-adds: the contraction of the stress and flux sums
        // is fixed, so S_PI and S_Q are the same bits with and without the
        // extension sensors; terms of a zero velocity component are skipped
        if (ia != 2) pxx = fma(vx * vx, fneq, pxx);
        if (ia != 2 && ib != 2) pxy = fma(vx * vy, fneq, pxy);
        if (ib != 2) pyy = fma(vy * vy, fneq, pyy);
        // raw third moments: sum v |v|^2/2 f^neq and sum v g^neq
        if (ia != 2) {
            qfx = fma(R(gh5_xi(ia) * 0.5 * (gh5_xi(ia) * gh5_xi(ia) + gh5_xi(ib) * gh5_xi(ib))), fneq, qfx);
            qgx = fma(vx, gneq, qgx);
        }
        if (ib != 2) {
            qfy = fma(R(gh5_xi(ib) * 0.5 * (gh5_xi(ia) * gh5_xi(ia) + gh5_xi(ib) * gh5_xi(ib))), fneq, qfy);
            qgy = fma(vy, gneq, qgy);
        }
    });
    const bool nonpos = !(eqmin > R(0)) || !(Tc > R(0)) || !(xlo > R(-1));
    if (!(xmax <= KlShortCut<R>::v) && !nonpos) {
        // rare: some population far from equilibrium (or NaN): the closed
        // form, one population at a time.  Cells with a positivity fault
        // skip it: their S_KL is +inf whatever the sums (on the paper's
        // supersonic Riemann problem No. 3 that is half of the cells)
        klf = R(0);
        klg = R(0);
        sfor25<25>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            const R w = R(gh5_w(i / 5) * gh5_w(i % 5));
            const R deq = deqv[i];
            const R feq = w * rho0 + deq;
            const R dgeq = gfac * (Tc * deq + tm1 * (w * rho0));
            const R geq = gfac * (w * rho0) + dgeq;
            klf += feq * kl_phi((fc[i] - deq) * rcp(feq));
            klg += geq * kl_phi((gc[i] - dgeq) * rcp(geq));
            __builtin_amdgcn_sched_barrier(0);
        });
    }
    // the total energy flux q = sum v (g^neq + |v|^2/2 f^neq) (S_Q), and the
    // heat fluxes relative to u: with sum f^neq = 0 and sum v f^neq = 0,
    // q_f = 1/2 sum |v - u|^2 (v - u) f^neq = Q_f - P u - (tr P / 2) u, and
    // q_g = sum (v - u) g^neq = Q_g - u sum g^neq
    const R qx = qfx + qgx, qy = qfy + qgy;
    {
        const R htr = R(0.5) * (pxx + pyy);
        qfx = qfx - fma(pxx, ux, fma(pxy, uy, htr * ux));
        qfy = qfy - fma(pxy, ux, fma(pyy, uy, htr * uy));
        qgx = fma(-ux, gsum, qgx);
        qgy = fma(-uy, gsum, qgy);
    }

    // q^neq through an opaque copy in both instantiations: the extension's use
    // of it must not change how the compiler contracts S_Q
    const R qxo = pin(qx), qyo = pin(qy);

    // ---- extension sensors (the rest of Table I with the g terms): a pass
    //      of their own on opaque copies (pin) of the moments and populations,
    //      so the base arithmetic is the same with and without them.  The QE
    //      parts of the dissipations, sum (h* - h^eq)_i L_i, are q . sum c_i v_i L_i
    //      with c_i = w_i (|v_i|^2/4 - 1) for f and w_i for g.
    R xv[EXT ? kNumExt : 1];
    if constexpr (EXT) {
        const R drho_p = pin(drho), rho_p = pin(rho), ux_p = pin(ux), uy_p = pin(uy), tm1_p = pin(tm1),
                rho0_p = pin(rho0), gfac_p = pin(gfac);
        const R Tc_p = R(1) + tm1_p;
        const ExtNeed need(a.x.mask);
        const bool needV = a.x.mask & 0x4u, needW = a.x.mask & 0x8u;
        ExtAcc<R> ef, eg;
        R vfx = R(0), vfy = R(0), wfx = R(0), wfy = R(0), vgx = R(0), vgy = R(0), wgx = R(0), wgy = R(0);
        // ln(g^eq/w) = ln((C_v - 1) T) + ln(f^eq/w) (g^eq = (C_v - 1) T f^eq)
        const R lgT = need.L ? ln1p_fast(gfac_p * Tc_p - R(1)) : R(0);
        d2q25_deq_pairs<R>(drho_p, rho_p, ux_p, uy_p, tm1_p, [&](int ia, int ib, R deq) {
            const int i = 5 * ia + ib;
            const R w = R(gh5_w(ia) * gh5_w(ib));
            const R iw = R(1.0 / (gh5_w(ia) * gh5_w(ib)));
            const R vx = R(gh5_xi(ia)), vy = R(gh5_xi(ib));
            const R d = pin(fc[i]), dg = pin(gc[i]);
            const R feq = w * rho0_p + deq, fneq = d - deq, x = fneq * rcp(feq);
            // c v of the entropy-flux sums: w (|v|^2/4 - 1) v for f, w v for g
            const double cf = gh5_w(ia) * gh5_w(ib) * (0.25 * (gh5_xi(ia) * gh5_xi(ia) + gh5_xi(ib) * gh5_xi(ib)) - 1.0);
            const double cg = gh5_w(ia) * gh5_w(ib);
            R ltf = R(0);                                                 // ln(f^eq/w)
            ext_add_vw(ef, need, needV, needW, fneq, x, w * rho0_p + d, (rho0_p - R(1)) + deq * iw, false, ltf,
                       R(cf * gh5_xi(ia)), R(cf * gh5_xi(ib)), vfx, vfy, wfx, wfy);
            const R dgeq = gfac_p * (Tc_p * deq + tm1_p * (w * rho0_p));
            const R geq = gfac_p * (w * rho0_p) + dgeq, gneq = dg - dgeq, y = gneq * rcp(geq);
            R ltg = ltf + lgT;                                            // ln(g^eq/w)
            ext_add_vw(eg, need, needV, needW, gneq, y, gfac_p * (w * rho0_p) + dg, R(0), true, ltg,
                       R(cg * gh5_xi(ia)), R(cg * gh5_xi(ib)), vgx, vgy, wgx, wgy);
        });
        const R inf = R(INFINITY);
        const bool fault_p = nonpos || !(fabs(klf) + fabs(klg + gsum) == fabs(klf) + fabs(klg + gsum));
        const R inv_mu = R(1.0 / a.mu);
        const R inv_tau1 = rho_p * Tc_p * inv_mu;
        const R d12 = inv_tau1 * (R(1) - R(a.prandtl));                  // 1/tau1 - 1/tau2
        const R qfx_p = pin(qfx), qfy_p = pin(qfy), qgx_p = pin(qgx), qgy_p = pin(qgy);
        auto alpha_dev = [](const ExtAcc<R>& e) {
            R dev = R(0);
            if (e.a1 != R(0)) {
                const R ia1 = rcp(R(0.5) * e.a1);
                const R r2 = R(-1.0 / 6.0) * e.a2 * ia1, r3 = R(1.0 / 12.0) * e.a3 * ia1,
                        r4 = R(-1.0 / 20.0) * e.a4 * ia1;
                dev = R(4) * r2 - R(16) * r2 * r2 + R(8) * r3 - R(80) * r2 * r3 + R(80) * r2 * r2 * r2 + R(16) * r4;
            }
            return fabs(dev);
        };
        // H(f) - H(f^eq) = sum f ln(f/f^eq) + sum f^neq ln(f^eq/w); the same for g
        const R hkf = pin(klf), hkg = pin(klg) + pin(gsum);
        xv[0] = fault_p ? inf : ef.kn + eg.kn;
        xv[1] = fault_p ? inf : fabs(hkf + ef.L) + fabs(hkg + eg.L);
        xv[2] = fault_p ? inf
                        : inv_tau1 * (ef.shkl + ef.L + eg.shkl + eg.L) -
                              d12 * (qfx_p * vfx + qfy_p * vfy + qgx_p * vgx + qgy_p * vgy);
        xv[3] = fault_p ? inf
                        : inv_tau1 * (ef.shkl + eg.shkl) - d12 * (qfx_p * wfx + qfy_p * wfy + qgx_p * wgx + qgy_p * wgy);
        xv[4] = fault_p ? inf : alpha_dev(ef) + alpha_dev(eg);
        const R pxx_p = pin(pxx), pxy_p = pin(pxy), pyy_p = pin(pyy);
        const R dxy = pxx_p - pyy_p;
        xv[5] = inv_mu * sqrt(R(0.5) * dxy * dxy + R(2) * pxy_p * pxy_p);
        const R hx = ux_p * pxx_p + uy_p * pxy_p, hy = ux_p * pxy_p + uy_p * pyy_p;
        xv[6] = sqrt(hx * hx + hy * hy);
        const R fx = qxo - hx, fy = qyo - hy;
        xv[7] = sqrt(fx * fx + fy * fy);
        // compression and strain with the model's second viscosity lambda =
        // -(R/C_v) mu and bulk viscosity eta = mu + lambda (D = 2; Sec. II.A.2,
        // eq. visc_bluk_1): sqrt(D)|tr P| / |2 mu + D lambda| and
        // |(1/2mu)[lambda/(D eta) tr(P) I - P]|_F
        const R trp = pxx_p + pyy_p;
        xv[8] = R(1.4142135623730951 / (2.0 * (a.mu - a.mu / a.cv))) * fabs(trp);
        const R cl = R(-1.0 / (2.0 * (a.cv - 1.0))), i2mu = R(0.5 / a.mu);
        const R exx = (cl * trp - pxx_p) * i2mu, eyy = (cl * trp - pyy_p) * i2mu, exy = -pxy_p * i2mu;
        xv[9] = sqrt(exx * exx + R(2) * exy * exy + eyy * eyy);
    }

    // ---- pass 2: f' = f - A div - (dt/tau1)(f - f^eq) + (dt/tau1 - dt/tau2)(f* - f^eq),
    //      f first, then g through the same buffer
    const AdvScale<R> adv(a);
    const R B1 = R(a.dt / a.mu) * rho * Tc;                // dt / tau1
    const R B12 = B1 * (R(1) - R(a.prandtl));              // dt / tau1 - dt / tau2
    const long long off = (long long)Y * nx + X;
    const long long poff = a.L.at(0, Y, X);
    __syncthreads();              // the staged f of the whole tile (pass 1 read registers only)
    auto update = [&](auto ic, R dfs, bool has_dfs) {
        constexpr int i = decltype(ic)::value;
        const R d = fc[i];
        const R c = fma(-B1, d - deqv[i], d);
        const R o = advect<R>(has_dfs ? fma(B12, dfs, c) : c, adv, lds + i * T::kPlane, rb, tx, d, i / 5, i % 5);
        if (active) put_pop<NTS>(fout + i * a.L.pp + poff, Store<S>::from_real(o));
    };
    // f* - f^eq = w (q_f . v)(|v|^2/4 - 1) is odd in v: population 24 - i
    // (velocity -v_i) takes -dfs_i bit for bit, and the rest population
    // none.  S_QE sums |f* - f^eq| and |g* - g^eq| = |w (q_g . v)| over the
    // populations: twice the sums over one of each pair
    R qe = R(0);
    update(std::integral_constant<int, 12>{}, R(0), false);
    sfor25<12>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        constexpr int ia = i / 5, ib = i % 5;
        const R dfs = R(gh5_w(ia) * gh5_w(ib) * (0.25 * (gh5_xi(ia) * gh5_xi(ia) + gh5_xi(ib) * gh5_xi(ib)) - 1.0)) *
                      q_dot_v(qfx, qfy, ia, ib);
        qe += fabs(dfs);
        update(ic, dfs, true);
        update(std::integral_constant<int, 24 - i>{}, -dfs, true);
    });
    // g itself is updated by d2q25_ddf_g_kernel from the cell state handed
    // over here
    sfor25<12>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        qe += fabs(R(gh5_w(i / 5) * gh5_w(i % 5)) * q_dot_v(qgx, qgy, i / 5, i % 5));
    });
    qe = R(2) * qe;
    if (active) {
        R* aux = static_cast<R*>(a.aux) + off;
        aux[0] = drho;
        aux[plane] = ux;
        aux[2 * plane] = uy;
        aux[3 * plane] = tm1;
        aux[4 * plane] = qgx;
        aux[5 * plane] = qgy;
    }

    // sum f ln(f/f^eq) = sum f^eq phi(x) (f and f^eq carry the same mass);
    // sum g ln(g/g^eq) = sum g^eq phi(y) + sum g^neq.  sum g^neq through an
    // opaque copy: it also feeds q_g, and whether the compiler fuses its
    // product into this sum must not depend on the extension sensors
    const R klsum = fabs(klf) + fabs(klg + pin(gsum));
    const bool fault = nonpos || !(klsum == klsum);
    const R s_kl = fault ? R(INFINITY) : klsum;
    // explicit multiply-adds: the same bits with and without the extension
    const R s_pi = sqrt_r(fma(pxx, pxx, fma(R(2) * pxy, pxy, pyy * pyy)));
    const R s_q = sqrt_r(fma(qxo, qxo, qyo * qyo));
    double acc[kNsums];
#pragma unroll
    for (int k = 0; k < kNsums; ++k) acc[k] = 0.0;
    if (active) {
        const R sv[5] = {s_kl, neq, s_pi, s_q, qe};
        LevelAcc lv;
#pragma unroll
        for (int s = 0; s < 5; ++s) {
            const R t0 = s < 4 ? R(a.thr[s][0]) : R(a.thr_qe[0]);
            const R t1 = s < 4 ? R(a.thr[s][1]) : R(a.thr_qe[1]);
            lv.add(sv[s], t0, t1);
        }
        if constexpr (EXT) {
            sfor25<kNumExt>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                if (a.x.plane[q] >= 0) sens[a.x.plane[q] * plane + off] = xv[q];
                if (a.mask & (1u << (kExtFlagShift + q))) lv.add(xv[q], R(a.x.thr[q][0]), R(a.x.thr[q][1]));
            });
        }
#pragma unroll
        for (int s = 0; s < 5; ++s) sens[s * plane + off] = sv[s];
        flags[off] = fault ? uint8_t(0x82) : uint8_t(lv.level());
        if (fault) atomicAdd(faults, 1ull);
        acc[0] = (double)drho;
        acc[1] = (double)jx;
        acc[2] = (double)jy;
        acc[3] = (double)dg0 + 0.5 * (double)m2;     // E - C_v rho0
        acc[4] = (double)s_kl;
        acc[5] = (double)neq;
        acc[6] = (double)s_pi;
        acc[7] = (double)s_q;
    }
    block_sums_n<NT / kWave>(acc, partials + (long long)blockIdx.x * kNsums);
}

// The g update of the double distribution: g is staged with its halo like
// f in d2q25_ddf_kernel, the cell state comes from that kernel's hand-over
// (drho, u, T - 1, q_g), and the collision and fluxes are those of f:
// g' = g - A div - (dt/tau1)(g - g^eq) + (dt/tau1 - dt/tau2)(g* - g^eq).
// Splitting the step here keeps the f kernel within two waves per SIMD
// without spilling registers.
template <typename S, int TX, int TY, bool EDGE = true, bool NTS = false>
__global__ __launch_bounds__(TX * TY) __attribute__((amdgpu_waves_per_eu(DdfGWaves<S>::v))) void d2q25_ddf_g_kernel(D2Q25Args a,
                                                         const typename Store<S>::raw* __restrict__ fin,
                                                         typename Store<S>::raw* __restrict__ fout)
{
    using R = typename Store<S>::real;
    using T = Tile<TX, TY>;
    constexpr int NG = 5;                      // planes per staged group
    constexpr int kStride = TileStage<S, TX, TY>::kStride;
    __shared__ R lds[2][NG * kStride];

    const int nx = a.nx, ny = a.ny;
    const long long plane = a.plane;
    int tile_x, tile_y;
    xcd_tile(a, tile_x, tile_y);
    const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
    const int X0 = tile_x * TX, Y0 = tile_y * TY;
    const int X = X0 + tx, Y = Y0 + ty;
    const bool active = !EDGE || (X < nx && Y < ny);     // EDGE: as in d2q25_kernel
    const TileStage<S, TX, TY> st(a, X0, Y0, tx, ty);
    constexpr int HR = TileStage<S, TX, TY>::HR;
    const int rb[5] = {T::rowbase(ty - 2), T::rowbase(ty - 1), T::rowbase(ty), T::rowbase(ty + 1),
                       T::rowbase(ty + 2)};
    const long long off = (long long)Y * nx + X;
    const long long poff = a.L.at(0, Y, X);

    // own-cell g values (registers), then g's stencil neighbours one velocity
    // group at a time through a double-buffered LDS tile, the next group's
    // halo in flight while this one is computed
    const typename Store<S>::raw* gin = fin + 25 * a.L.pp;
    R gc[25];
    sfor25<25>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        gc[i] = Store<S>::to_real(gin[i * a.L.pp + st.own]);
    });
    R vh[NG][HR], vc[NG];
    st.template load<NG>(gin, a.L.pp, 0, vh, vc);

    // the cell state from the f kernel (own cell only; ghost threads stage)
    R drho = R(0), ux = R(0), uy = R(0), tm1 = R(0), qgx = R(0), qgy = R(0);
    if (active) {
        const R* aux = static_cast<const R*>(a.aux) + off;
        drho = aux[0];
        ux = aux[plane];
        uy = aux[2 * plane];
        tm1 = aux[3 * plane];
        qgx = aux[4 * plane];
        qgy = aux[5 * plane];
    }
    const R rho0 = R(a.rho0);
    const R gfac = R(a.cv) - R(1);
    const R rho = rho0 + drho;
    const R Tc = R(1) + tm1;
    const AdvScale<R> adv(a);
    const R B1 = R(a.dt / a.mu) * rho * Tc;                // dt / tau1
    const R B12 = B1 * (R(1) - R(a.prandtl));              // dt / tau1 - dt / tau2
    const Deq25<R> eq(drho, rho, ux, uy, tm1);

    st.template write<NG, 0>(lds[0], gc, vh, vc);
    __syncthreads();
    sfor25<5>([&](auto gcn) {
        constexpr int g = decltype(gcn)::value;
        if constexpr (g + 1 < 5) st.template load<NG>(gin, a.L.pp, NG * (g + 1), vh, vc);
        const R* buf = lds[g & 1];
        eq.template group<g>([&](int ia, int ib, R deq) {
            const int i = 5 * ia + ib;
            const R w = R(gh5_w(ia) * gh5_w(ib));
            const R vx = R(gh5_xi(ia)), vy = R(gh5_xi(ib));
            const R dg = gc[i];
            const R gneq = dg - gfac * (Tc * deq + tm1 * (w * rho0));
            const R dgs = w * (qgx * vx + qgy * vy);
            const R o = advect<R>(fma(B12, dgs, fma(-B1, gneq, dg)), adv, buf + ib * kStride, rb, tx, dg, ia, ib);
            if (active) put_pop<NTS>(fout + (25 + i) * a.L.pp + poff, Store<S>::from_real(o));
        });
        if constexpr (g + 1 < 5) {
            st.template write<NG, NG * (g + 1)>(lds[(g + 1) & 1], gc, vh, vc);
            __syncthreads();
        }
    });
}

template <typename S, int TX, int TY>
static hipError_t launch_ddf_tile(const D2Q25Args& a, const void* fin, void* fout, void* sens,
                                  uint8_t* flags, double* partials, unsigned long long* faults,
                                  hipStream_t s)
{
    // the g kernel writes no partial sums: it runs on a tile grid of its own
    constexpr int GX = sizeof(typename Store<S>::real) == 4 ? LKS_DDF_G_TX : TX;
    constexpr int GY = sizeof(typename Store<S>::real) == 4 ? LKS_DDF_G_TY : TY;
    using raw = typename Store<S>::raw;
    using R = typename Store<S>::real;
    if (a.tile_x != TX || a.tile_y != TY) return hipErrorInvalidValue;
    if (!a.aux) return hipErrorInvalidValue;
    // the same EDGE form with and without the extension sensors (as above);
    // the non-temporal stores on whole FP32 tiles whose rows are whole
    // 128-byte lines only (on the f kernel's 16-float rows they wrote 717
    // instead of 614 MB per step at 2048^2)
    const bool whole = a.nx % TX == 0 && a.ny % TY == 0;
    constexpr bool kNT = std::is_same<S, float>::value && TX * sizeof(R) >= 128;
    const bool nt = kNT && whole && a.nt_stores;
    if (a.x.mask && nt)
        d2q25_ddf_kernel<S, TX, TY, true, false, kNT><<<dim3(a.nblocks), dim3(TX * TY), 0, s>>>(
            a, (const raw*)fin, (raw*)fout, (R*)sens, flags, partials, faults);
    else if (a.x.mask && whole)
        d2q25_ddf_kernel<S, TX, TY, true, false><<<dim3(a.nblocks), dim3(TX * TY), 0, s>>>(
            a, (const raw*)fin, (raw*)fout, (R*)sens, flags, partials, faults);
    else if (a.x.mask)
        d2q25_ddf_kernel<S, TX, TY, true, true><<<dim3(a.nblocks), dim3(TX * TY), 0, s>>>(
            a, (const raw*)fin, (raw*)fout, (R*)sens, flags, partials, faults);
    else if (nt)
        d2q25_ddf_kernel<S, TX, TY, false, false, kNT><<<dim3(a.nblocks), dim3(TX * TY), 0, s>>>(
            a, (const raw*)fin, (raw*)fout, (R*)sens, flags, partials, faults);
    else if (whole)
        d2q25_ddf_kernel<S, TX, TY, false, false><<<dim3(a.nblocks), dim3(TX * TY), 0, s>>>(
            a, (const raw*)fin, (raw*)fout, (R*)sens, flags, partials, faults);
    else
        d2q25_ddf_kernel<S, TX, TY, false, true><<<dim3(a.nblocks), dim3(TX * TY), 0, s>>>(
            a, (const raw*)fin, (raw*)fout, (R*)sens, flags, partials, faults);
    if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
    D2Q25Args ag = a;
    ag.tile_x = GX;
    ag.tile_y = GY;
    ag.tiles_x = (a.nx + GX - 1) / GX;
    ag.tiles_y = (a.ny + GY - 1) / GY;
    ag.nblocks = ag.tiles_x * ag.tiles_y;
    const bool gwhole = a.nx % GX == 0 && a.ny % GY == 0;
    constexpr bool kGNT = std::is_same<S, float>::value && GX * sizeof(R) >= 128;
    if (kGNT && gwhole && a.nt_stores)
        d2q25_ddf_g_kernel<S, GX, GY, false, kGNT><<<dim3(ag.nblocks), dim3(GX * GY), 0, s>>>(ag, (const raw*)fin, (raw*)fout);
    else if (gwhole)
        d2q25_ddf_g_kernel<S, GX, GY, false><<<dim3(ag.nblocks), dim3(GX * GY), 0, s>>>(ag, (const raw*)fin, (raw*)fout);
    else
        d2q25_ddf_g_kernel<S, GX, GY><<<dim3(ag.nblocks), dim3(GX * GY), 0, s>>>(ag, (const raw*)fin, (raw*)fout);
    return hipGetLastError();
}

template <typename S, int TX, int TY>
static hipError_t launch_tile(const D2Q25Args& a, const void* fin, void* fout, void* sens, uint8_t* flags,
                              double* partials, unsigned long long* faults, hipStream_t s)
{
    using raw = typename Store<S>::raw;
    using R = typename Store<S>::real;
    if (a.tile_x != TX || a.tile_y != TY) return hipErrorInvalidValue;
    // with and without the extension sensors the same EDGE form runs, so the
    // base outputs stay the same bits; the non-temporal stores on whole FP32
    // tiles of whole 128-byte rows only
    const bool whole = a.nx % TX == 0 && a.ny % TY == 0;
    constexpr bool kNT = std::is_same<S, float>::value && TX * sizeof(R) >= 128;
    const bool nt = kNT && whole && a.nt_stores;
    if (a.x.mask && nt)
        d2q25_kernel<S, TX, TY, true, false, kNT><<<dim3(a.nblocks), dim3(TX * TY), 0, s>>>(
            a, (const raw*)fin, (raw*)fout, (R*)sens, flags, partials, faults);
    else if (a.x.mask && whole)
        d2q25_kernel<S, TX, TY, true, false><<<dim3(a.nblocks), dim3(TX * TY), 0, s>>>(
            a, (const raw*)fin, (raw*)fout, (R*)sens, flags, partials, faults);
    else if (a.x.mask)
        d2q25_kernel<S, TX, TY, true, true><<<dim3(a.nblocks), dim3(TX * TY), 0, s>>>(
            a, (const raw*)fin, (raw*)fout, (R*)sens, flags, partials, faults);
    else if (nt)
        d2q25_kernel<S, TX, TY, false, false, kNT><<<dim3(a.nblocks), dim3(TX * TY), 0, s>>>(
            a, (const raw*)fin, (raw*)fout, (R*)sens, flags, partials, faults);
    else if (whole)
        d2q25_kernel<S, TX, TY, false, false><<<dim3(a.nblocks), dim3(TX * TY), 0, s>>>(
            a, (const raw*)fin, (raw*)fout, (R*)sens, flags, partials, faults);
    else
        d2q25_kernel<S, TX, TY, false, true><<<dim3(a.nblocks), dim3(TX * TY), 0, s>>>(
            a, (const raw*)fin, (raw*)fout, (R*)sens, flags, partials, faults);
    return hipGetLastError();
}

hipError_t launch_d2q25(int dtype, const D2Q25Args& a, const void* fin, void* fout, void* sens,
                        uint8_t* flags, double* partials, unsigned long long* faults, hipStream_t s)
{
    if (a.model == 1) {
        switch (dtype) {
        case 0: return launch_ddf_tile<double, 16, 4>(a, fin, fout, sens, flags, partials, faults, s);
        case 1: return launch_ddf_tile<float, LKS_DDF_TX, LKS_DDF_TY>(a, fin, fout, sens, flags, partials, faults, s);
        default: return hipErrorInvalidValue;
        }
    }
    switch (dtype) {
    case 0: return launch_tile<double, 32, 2>(a, fin, fout, sens, flags, partials, faults, s);
    case 1: return launch_tile<float, LKS_Q25_TX, LKS_Q25_TY>(a, fin, fout, sens, flags, partials, faults, s);
    default: return hipErrorInvalidValue;
    }
}

// tile shape the launcher expects for a storage type and model
void d2q25_tile_shape(int dtype, int model, int* tx, int* ty)
{
    if (model == 1) {
        *tx = dtype == 0 ? 16 : LKS_DDF_TX;
        *ty = dtype == 0 ? 4 : LKS_DDF_TY;
        return;
    }
    *tx = dtype == 0 ? 32 : LKS_Q25_TX;
    *ty = dtype == 0 ? 2 : LKS_Q25_TY;
}

// ---------------------------------------------------------------------------
// Equilibrium initialiser and moment readout (one thread per cell, FP64 math)
// ---------------------------------------------------------------------------
template <typename S>
__global__ __launch_bounds__(kBlock) void d2q25_init_kernel(long long n, PopLayout L, double rho0, const double* __restrict__ rho,
                                                       const double* __restrict__ ux,
                                                       const double* __restrict__ uy,
                                                       const double* __restrict__ T,
                                                       typename Store<S>::raw* __restrict__ pop)
{
    const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (c >= n) return;
    const double r = rho[c];
    d2q25_deq<double>(r - rho0, r, ux[c], uy[c], T[c] - 1.0, [&](int ia, int ib, double deq) {
        pop[L.cell(5 * ia + ib, c)] = Store<S>::from_real((typename Store<S>::real)deq);
    });
}

template <typename S>
__global__ __launch_bounds__(kBlock) void d2q25_moments_kernel(long long n, PopLayout L, double rho0,
                                                          const typename Store<S>::raw* __restrict__ pop,
                                                          double* __restrict__ rho, double* __restrict__ ux,
                                                          double* __restrict__ uy, double* __restrict__ T)
{
    const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (c >= n) return;
    double drho = 0.0, jx = 0.0, jy = 0.0, edev = 0.0;
#pragma unroll
    for (int i = 0; i < 25; ++i) {
        const double d = (double)Store<S>::to_real(pop[L.cell(i, c)]);
        const double vx = gh5_xi(i / 5), vy = gh5_xi(i % 5);
        drho += d;
        jx += vx * d;
        jy += vy * d;
        edev += 0.5 * (vx * vx + vy * vy) * d;
    }
    const double r = rho0 + drho;
    const double u = jx / r, v = jy / r;
    rho[c] = r;
    ux[c] = u;
    uy[c] = v;
    if (T) T[c] = 1.0 + (edev - drho) / r - 0.5 * (u * u + v * v);
}

// double distribution: f^eq and g^eq = (C_v - 1) T f^eq as deviations
template <typename S>
__global__ __launch_bounds__(kBlock) void d2q25_ddf_init_kernel(long long n, PopLayout L, double rho0, double cv,
                                                           const double* __restrict__ rho,
                                                           const double* __restrict__ ux,
                                                           const double* __restrict__ uy,
                                                           const double* __restrict__ T,
                                                           typename Store<S>::raw* __restrict__ pop)
{
    const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (c >= n) return;
    const double r = rho[c], t = T[c];
    d2q25_deq<double>(r - rho0, r, ux[c], uy[c], t - 1.0, [&](int ia, int ib, double deq) {
        const int i = 5 * ia + ib;
        const double w = gh5_w(ia) * gh5_w(ib);
        pop[L.cell(i, c)] = Store<S>::from_real((typename Store<S>::real)deq);
        const double dgeq = (cv - 1.0) * (t * deq + (t - 1.0) * w * rho0);
        pop[L.cell(25 + i, c)] = Store<S>::from_real((typename Store<S>::real)dgeq);
    });
}

template <typename S>
__global__ __launch_bounds__(kBlock) void d2q25_ddf_moments_kernel(long long n, PopLayout L, double rho0, double cv,
                                                              const typename Store<S>::raw* __restrict__ pop,
                                                              double* __restrict__ rho,
                                                              double* __restrict__ ux,
                                                              double* __restrict__ uy,
                                                              double* __restrict__ T)
{
    const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (c >= n) return;
    double drho = 0.0, jx = 0.0, jy = 0.0, m2 = 0.0, dg0 = 0.0;
#pragma unroll
    for (int i = 0; i < 25; ++i) {
        const double d = (double)Store<S>::to_real(pop[L.cell(i, c)]);
        const double vx = gh5_xi(i / 5), vy = gh5_xi(i % 5);
        drho += d;
        jx += vx * d;
        jy += vy * d;
        m2 += (vx * vx + vy * vy) * d;
        dg0 += (double)Store<S>::to_real(pop[L.cell(25 + i, c)]);
    }
    const double r = rho0 + drho;
    const double u = jx / r, v = jy / r;
    rho[c] = r;
    ux[c] = u;
    uy[c] = v;
    if (T) T[c] = 1.0 + ((dg0 + 0.5 * m2 - cv * drho) / r - 0.5 * (u * u + v * v)) / cv;
}

hipError_t launch_d2q25_ddf_init(int dtype, long long n, const PopLayout& L, double rho0, double cv, const double* rho,
                                 const double* ux, const double* uy, const double* T, void* pop,
                                 hipStream_t s)
{
    const dim3 grid((unsigned)((n + kBlock - 1) / kBlock)), block(kBlock);
    switch (dtype) {
    case 0: d2q25_ddf_init_kernel<double><<<grid, block, 0, s>>>(n, L, rho0, cv, rho, ux, uy, T, (double*)pop); break;
    case 1: d2q25_ddf_init_kernel<float><<<grid, block, 0, s>>>(n, L, rho0, cv, rho, ux, uy, T, (float*)pop); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_d2q25_ddf_moments(int dtype, long long n, const PopLayout& L, double rho0, double cv, const void* pop,
                                    double* rho, double* ux, double* uy, double* T, hipStream_t s)
{
    const dim3 grid((unsigned)((n + kBlock - 1) / kBlock)), block(kBlock);
    switch (dtype) {
    case 0: d2q25_ddf_moments_kernel<double><<<grid, block, 0, s>>>(n, L, rho0, cv, (const double*)pop, rho, ux, uy, T); break;
    case 1: d2q25_ddf_moments_kernel<float><<<grid, block, 0, s>>>(n, L, rho0, cv, (const float*)pop, rho, ux, uy, T); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_d2q25_init(int dtype, long long n, const PopLayout& L, double rho0, const double* rho, const double* ux,
                             const double* uy, const double* T, void* pop, hipStream_t s)
{
    const dim3 grid((unsigned)((n + kBlock - 1) / kBlock)), block(kBlock);
    switch (dtype) {
    case 0: d2q25_init_kernel<double><<<grid, block, 0, s>>>(n, L, rho0, rho, ux, uy, T, (double*)pop); break;
    case 1: d2q25_init_kernel<float><<<grid, block, 0, s>>>(n, L, rho0, rho, ux, uy, T, (float*)pop); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_d2q25_moments(int dtype, long long n, const PopLayout& L, double rho0, const void* pop, double* rho,
                                double* ux, double* uy, double* T, hipStream_t s)
{
    const dim3 grid((unsigned)((n + kBlock - 1) / kBlock)), block(kBlock);
    switch (dtype) {
    case 0: d2q25_moments_kernel<double><<<grid, block, 0, s>>>(n, L, rho0, (const double*)pop, rho, ux, uy, T); break;
    case 1: d2q25_moments_kernel<float><<<grid, block, 0, s>>>(n, L, rho0, (const float*)pop, rho, ux, uy, T); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

} // namespace lks
