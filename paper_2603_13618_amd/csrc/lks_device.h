// lks_device.h -- device-side building blocks shared by the gfx950 kernels:
// storage conversions, packed vector loads/stores, the KL integrand and
// wave64 FP64 reductions.  HIP only; included by the kernel sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

// Occupancy hint for the cell kernels: minimum waves per SIMD the register
// allocation must allow (0 = let the compiler decide).
#ifndef LKS_WAVES_PER_EU
#define LKS_WAVES_PER_EU 0
#endif
#if LKS_WAVES_PER_EU > 0
#define LKS_CELL_KERNEL_ATTR __attribute__((amdgpu_waves_per_eu(LKS_WAVES_PER_EU)))
#else
#define LKS_CELL_KERNEL_ATTR
#endif

// Rows of populations the D2Q9 kernel keeps in flight ahead of the row it
// computes.
#ifndef LKS_D2Q9_PREFETCH
#define LKS_D2Q9_PREFETCH 1
#endif
// 1 = the fused D2Q9 step stages the next row through LDS with direct
// global->LDS loads where a lane's cells span whole dwords (4, 8 or 16 bytes).
#ifndef LKS_D2Q9_LDS_STAGE
#define LKS_D2Q9_LDS_STAGE 1
#endif
// 1 = a scheduling barrier between the cells a thread updates, so the
// compiler does not interleave them (shorter live ranges, fewer VGPRs).
#ifndef LKS_CELL_SCHED_BARRIER
#define LKS_CELL_SCHED_BARRIER 0
#endif
#if LKS_CELL_SCHED_BARRIER
#define LKS_CELL_BARRIER() __builtin_amdgcn_sched_barrier(0)
#else
#define LKS_CELL_BARRIER() ((void)0)
#endif
// Non-temporal loads for the population planes (read once per step).
#ifndef LKS_NT_LOADS
#define LKS_NT_LOADS 0
#endif

namespace lks {

constexpr int kWave = 64;
constexpr int kBlock = 256;          // 4 waves per workgroup
constexpr int kNsums = 8;

// ---------------------------------------------------------------------------
// Storage types.  Populations are stored as deviations d = f - w*rho0; the
// 16-bit formats are raw bit patterns (uint16_t) to keep loads plain.
// ---------------------------------------------------------------------------
struct bf16_t { uint16_t bits; };
struct f16_t { uint16_t bits; };

// The 16-bit forms store the FP32 result rounded to nearest even.  The
// conversion must start from that FP32 value: left alone, the compiler folds
// a float->half conversion into the FMA that produced the value
// (v_fma_mix*), rounding once from the exact product-sum, which differs from
// rounding the FP32 result on exact FP16 ties.  pin_f32 makes the value
// opaque (an empty asm on its register), so the conversion is a separate
// instruction (v_cvt_*, round to nearest even in the default mode).
__device__ __forceinline__ float pin_f32(float f)
{
    asm("" : "+v"(f));
    return f;
}
// the same barrier for any register-sized value (FP64 takes a register pair)
template <typename T> __device__ __forceinline__ T pin(T v)
{
    asm("" : "+v"(v));
    return v;
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) { return __builtin_bit_cast(uint16_t, (__bf16)pin_f32(f)); }
__device__ __forceinline__ float f16_to_f32(uint16_t h) { return (float)__builtin_bit_cast(_Float16, h); }
__device__ __forceinline__ uint16_t f32_to_f16_rne(float f) { return __builtin_bit_cast(uint16_t, (_Float16)pin_f32(f)); }

template <typename S> struct Store;
template <> struct Store<double> {
    using raw = double;
    using real = double;
    __device__ static double to_real(raw v) { return v; }
    __device__ static raw from_real(double v) { return v; }
};
template <> struct Store<float> {
    using raw = float;
    using real = float;
    __device__ static float to_real(raw v) { return v; }
    __device__ static raw from_real(float v) { return v; }
};
template <> struct Store<bf16_t> {
    using raw = uint16_t;
    using real = float;
    __device__ static float to_real(raw v) { return bf16_to_f32(v); }
    __device__ static raw from_real(float v) { return f32_to_bf16_rne(v); }
};
template <> struct Store<f16_t> {
    using raw = uint16_t;
    using real = float;
    __device__ static float to_real(raw v) { return f16_to_f32(v); }
    __device__ static raw from_real(float v) { return f32_to_f16_rne(v); }
};

// VEC consecutive elements as one aligned memory operation
template <typename T, int VEC> struct alignas(sizeof(T) * VEC) Pack { T v[VEC]; };

// store of a pack, with the non-temporal hint when NT (for outputs that no
// cache can hold until they are read again)
template <typename T, int VEC, bool NT = false>
__device__ __forceinline__ void store_raw_pack(T* __restrict__ p, const Pack<T, VEC>& pk)
{
    constexpr int bytes = (int)sizeof(T) * VEC;
    if constexpr (!NT) {
        *reinterpret_cast<Pack<T, VEC>*>(p) = pk;
    } else if constexpr (bytes == 16) {
        using V = __attribute__((ext_vector_type(4))) unsigned int;
        __builtin_nontemporal_store(__builtin_bit_cast(V, pk), reinterpret_cast<V*>(p));
    } else if constexpr (bytes == 8) {
        using V = __attribute__((ext_vector_type(2))) unsigned int;
        __builtin_nontemporal_store(__builtin_bit_cast(V, pk), reinterpret_cast<V*>(p));
    } else if constexpr (bytes == 4) {
        __builtin_nontemporal_store(__builtin_bit_cast(unsigned int, pk), reinterpret_cast<unsigned int*>(p));
    } else if constexpr (bytes == 2) {
        __builtin_nontemporal_store(__builtin_bit_cast(unsigned short, pk), reinterpret_cast<unsigned short*>(p));
    } else {
        __builtin_nontemporal_store(__builtin_bit_cast(unsigned char, pk), reinterpret_cast<unsigned char*>(p));
    }
}

template <typename S, int VEC>
__device__ __forceinline__ void load_vec(const typename Store<S>::raw* __restrict__ p,
                                         typename Store<S>::real (&out)[VEC])
{
    using raw = typename Store<S>::raw;
#if LKS_NT_LOADS
    constexpr int bytes = (int)sizeof(raw) * VEC;
    Pack<raw, VEC> pk;
    if constexpr (bytes == 16) {
        using V = __attribute__((ext_vector_type(4))) unsigned int;
        pk = __builtin_bit_cast(Pack<raw, VEC>, __builtin_nontemporal_load(reinterpret_cast<const V*>(p)));
    } else if constexpr (bytes == 8) {
        using V = __attribute__((ext_vector_type(2))) unsigned int;
        pk = __builtin_bit_cast(Pack<raw, VEC>, __builtin_nontemporal_load(reinterpret_cast<const V*>(p)));
    } else {
        pk = *reinterpret_cast<const Pack<raw, VEC>*>(p);
    }
#else
    const Pack<raw, VEC> pk = *reinterpret_cast<const Pack<raw, VEC>*>(p);
#endif
#pragma unroll
    for (int k = 0; k < VEC; ++k) out[k] = Store<S>::to_real(pk.v[k]);
}

template <typename S, int VEC, bool NT = false>
__device__ __forceinline__ void store_vec(typename Store<S>::raw* __restrict__ p,
                                          const typename Store<S>::real (&in)[VEC])
{
    using raw = typename Store<S>::raw;
    Pack<raw, VEC> pk;
    constexpr bool half = std::is_same<S, bf16_t>::value || std::is_same<S, f16_t>::value;
    if constexpr (half && VEC % 2 == 0) {
        // two values per packed conversion
        using F2 = __attribute__((ext_vector_type(2))) float;
        using H2 = __attribute__((ext_vector_type(2)))
            typename std::conditional<std::is_same<S, bf16_t>::value, __bf16, _Float16>::type;
#pragma unroll
        for (int k = 0; k < VEC; k += 2) {
            const H2 h = __builtin_convertvector(F2{pin_f32(in[k]), pin_f32(in[k + 1])}, H2);
            const uint32_t u = __builtin_bit_cast(uint32_t, h);
            pk.v[k] = (uint16_t)(u & 0xffffu);
            pk.v[k + 1] = (uint16_t)(u >> 16);
        }
    } else {
#pragma unroll
        for (int k = 0; k < VEC; ++k) pk.v[k] = Store<S>::from_real(in[k]);
    }
    store_raw_pack<raw, VEC, NT>(p, pk);
}

template <typename T, int VEC, bool NT = false>
__device__ __forceinline__ void store_pack(T* __restrict__ p, const T (&in)[VEC])
{
    Pack<T, VEC> pk;
#pragma unroll
    for (int k = 0; k < VEC; ++k) pk.v[k] = in[k];
    store_raw_pack<T, VEC, NT>(p, pk);
}

// ---------------------------------------------------------------------------
// Arithmetic helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float log1p_r(float x) { return log1pf(x); }
__device__ __forceinline__ double log1p_r(double x) { return log1p(x); }

// KL integrand phi(x) = (1+x) ln(1+x) - x, so that f ln(f/feq) - f + feq =
// feq * phi(fneq/feq) = fneq * x * p(x) with x = fneq/feq and p(x) = phi(x)/x^2.
// The FP64 multiply-adds here are explicit fma: left to contraction, whether
// a multiply and an add fuse depends on the basic blocks around the inlined
// code, which differ between kernels, and the sensors are to be the same bits
// in every kernel that computes them.  (The FP32 series is left to
// contraction: written as fma it costs the D2Q25 kernel 18 registers and a
// wave per SIMD, and its bits agree between kernels as written.)
// Near 0 the closed form cancels; there the Taylor series
// p(x) = sum_{n>=2} (-1)^n x^(n-2) / (n(n-1)) is used for |x| <= KlCut:
// truncated after n = 7 in FP32 (relative truncation 2 x^6/56 < 4e-8 at
// |x| = 0.1) and after n = 9 in FP64 (2 x^8/90 < 3e-18 at |x| = 0.01).
template <typename R> struct KlCut;
template <> struct KlCut<float> { static constexpr float v = 0.1f; };
template <> struct KlCut<double> { static constexpr double v = 0.01; };

__device__ __forceinline__ float kl_series(float x)
{
    float p = -1.0f / 42.0f;
    p = p * x + 1.0f / 30.0f;
    p = p * x + -1.0f / 20.0f;
    p = p * x + 1.0f / 12.0f;
    p = p * x + -1.0f / 6.0f;
    p = p * x + 0.5f;
    return p;
}

__device__ __forceinline__ double kl_series(double x)
{
    double p = -1.0 / 72.0;
    p = fma(p, x, 1.0 / 56.0);
    p = fma(p, x, -1.0 / 42.0);
    p = fma(p, x, 1.0 / 30.0);
    p = fma(p, x, -1.0 / 20.0);
    p = fma(p, x, 1.0 / 12.0);
    p = fma(p, x, -1.0 / 6.0);
    p = fma(p, x, 0.5);
    return p;
}

// The D2Q9 cell update's first try: in FP32 the series truncated after
// n = 5 for |x| <= 0.03 (relative truncation 2 x^4/30 < 5.4e-8), two
// multiply-adds per population fewer than kl_series; cells with a larger
// |x| take kl_phi.  On the smooth and shear-layer workloads every cell has
// |x| < 0.02, so the fallback never runs there.  FP64 keeps kl_series.
template <typename R> struct KlShortCut;
template <> struct KlShortCut<float> { static constexpr float v = 0.03f; };
template <> struct KlShortCut<double> { static constexpr double v = KlCut<double>::v; };
__device__ __forceinline__ float kl_series_short(float x)
{
    float p = -1.0f / 20.0f;
    p = p * x + 1.0f / 12.0f;
    p = p * x + -1.0f / 6.0f;
    p = p * x + 0.5f;
    return p;
}
__device__ __forceinline__ double kl_series_short(double x) { return kl_series(x); }

// Refinement level of a cell: per enabled sensor k, [s_k > t1_k] +
// [s_k > t2_k], the maximum over k.  With t1 <= t2 (checked at creation, and
// kept by the rounding to FP32) that maximum is 2 when some s_k > t2_k, else
// 1 when some s_k > t1_k: the comparisons only OR lane masks, and one select
// gives the level.  A NaN sensor compares false, as in the sum of the two.
struct LevelAcc {
    bool any1 = false, any2 = false;
    template <typename R> __device__ __forceinline__ void add(R s, R t1, R t2)
    {
        any1 = any1 | (s > t1);
        any2 = any2 | (s > t2);
    }
    __device__ __forceinline__ int level() const { return any2 ? 2 : (any1 ? 1 : 0); }
};

// Square root of a sensor norm: in FP32 the hardware instruction
// (v_sqrt_f32, within 1 ulp; the correctly rounded library sequence adds
// about 14 instructions per call), in FP64 the library's sqrt.
__device__ __forceinline__ float sqrt_r(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double sqrt_r(double x) { return sqrt(x); }

// phi(x) on either branch
template <typename R>
__device__ __forceinline__ R kl_phi(R x)
{
    if (fabs(x) <= KlCut<R>::v) return x * x * kl_series(x);
    return fma(R(1) + x, log1p_r(x), -x);
}

// derivative phi'(x) = ln(1+x) (used by the adjoint seed)
template <typename R>
__device__ __forceinline__ R kl_dphi(R x) { return log1p_r(x); }

// ---------------------------------------------------------------------------
// Extended sensors: the rest of Table I on the f distribution, computed in
// the same pass when a kernel is instantiated with them.  Order of the
// values (and of the ABI's extension bits):
//   0 Knudsen      sum |f^neq/f^eq|                      (eq. sensor-Knudsen-kin_f)
//   1 relative H   |H(f) - H(f^eq)|, H = sum f ln(f/w)   (eq. Hneq-sensor)
//   2 H dissipation   -sum Omega ln(f/w)                 (eq. Dissip-H-sensor)
//   3 KL dissipation  -sum Omega ln(f/f^eq)              (eq. Dissip-HKL-sensor)
//   4 entropic estimate |2 - alpha_f|, printed polynomial (eqs. alpha-polynomial-1/2)
//   5 rate of shear |(1/mu)[(tr P/D) I - P]|             (eq. sensor-S-kin)
//   6 viscous heating |u . P|                             (eq. sensor-qH-kin)
//   7 Fourier flux |q^neq - u . P| (D2Q25)               (eq. sensor-qF-kin-ryk, g = 0)
//   8 rate of compression sqrt(D)|tr P|/(2 mu) (D2Q9, lambda = 0)   (eq. sensor-C-kin)
//   9 rate of strain |P|/(2 mu) (D2Q9, lambda = 0)      (eq. sensor-E-kin)
// with Omega_i = -(f_i - f^eq_i)/tau (BGK), P = sum v v f^neq.
// Cancellation-free forms (sum_i f^neq_i = 0 because f^eq carries the cell's
// own mass): H(f) - H(f^eq) = S_KL + sum f^neq ln(f^eq/w) and
// -sum Omega ln(f/w) = (1/tau) [sum f^neq ln(1 + x) + sum f^neq ln(f^eq/w)],
// x = f^neq/f^eq; 2 - alpha is evaluated directly, not as a difference.
// ---------------------------------------------------------------------------
constexpr int kNumExt = 10;

// ln(1 + t) for the extension sensors.  FP32: ln(1 + t) = 2 atanh(u),
// u = t / (2 + t), as the odd series to u^11 for t in [-0.4, 0.5] (|u| <= 1/4,
// relative truncation u^12 / 13 < 5e-9, one reciprocal and six FMAs), else the
// hardware base-2 logarithm of 1 + t (ln is not small there, so its absolute
// accuracy suffices).  FP64: the library log1p.
__device__ __forceinline__ float ln1p_fast(float t)
{
    const float u = t * rcp(2.0f + t);
    const float u2 = u * u;
    float p = 2.0f / 11.0f;
    p = p * u2 + 2.0f / 9.0f;
    p = p * u2 + 2.0f / 7.0f;
    p = p * u2 + 2.0f / 5.0f;
    p = p * u2 + 2.0f / 3.0f;
    p = p * u2 + 2.0f;
    const float direct = __builtin_amdgcn_logf(1.0f + t) * 0.69314718055994531f;
    return (t >= -0.4f && t <= 0.5f) ? u * p : direct;
}
__device__ __forceinline__ double ln1p_fast(double t) { return log1p(t); }

// which of the costly per-population sums a launch needs (wave-uniform, so
// the guards are scalar branches): the sum of f^neq ln(f^eq/w) (relative H,
// H dissipation), of f^neq ln(1 + x) (both dissipations), the alpha moments
struct ExtNeed {
    bool L, S, A;
    __device__ __forceinline__ explicit ExtNeed(unsigned m)
        : L(m & 0x6u), S(m & 0xCu), A(m & 0x10u) {}
};

template <typename R> struct ExtAcc {
    R kn = R(0), L = R(0), shkl = R(0), a1 = R(0), a2 = R(0), a3 = R(0), a4 = R(0);
    // one population: its non-equilibrium part, x = fneq/feq, f itself and
    // t = f^eq/w - 1
    // The inputs are taken through pin() so that nothing computed here is
    // shared with (and changes the contraction of) the base arithmetic.
    __device__ __forceinline__ void add(const ExtNeed& need, R fneq_, R x_, R f_, R t_)
    {
        const R fneq = pin(fneq_), x = pin(x_), f = pin(f_), t = pin(t_);
        kn += fabs(x);
        if (need.L) L += fneq * ln1p_fast(t);
        if (need.S) shkl += fneq * ln1p_fast(x);
        if (need.A) {
            const R y = fneq * rcp(f);             // f^neq / f
            const R t1 = fneq * y, t2 = t1 * y, t3 = t2 * y;
            a1 += t1;
            a2 += t2;
            a3 += t3;
            a4 += t3 * y;
        }
    }
};

// Finish the extended sensors of one cell.  kl = S_KL, inv_tau = 1/tau,
// inv_mu = 1/mu; P components, velocity and (D2Q25) q^neq; d2q25 selects the
// lattice-specific entries (Fourier flux there, compression and strain on
// D2Q9).  A positivity fault makes the five log/ratio sensors +inf.  The
// stress components are taken through pin() so that no product here is
// shared with the base sensors' arithmetic (which would change how the
// compiler contracts S_PI and make it differ by an ulp with the extension on).
template <typename R>
__device__ __forceinline__ void ext_finish(const ExtAcc<R>& e, R kl, bool fault, R inv_tau, R inv_mu,
                                           R pxx_, R pxy_, R pyy_, R ux, R uy, R qx, R qy, bool d2q25,
                                           R (&out)[kNumExt])
{
    const R pxx = pin(pxx_), pxy = pin(pxy_), pyy = pin(pyy_);
    const R inf = R(INFINITY);
    out[0] = fault ? inf : e.kn;
    out[1] = fault ? inf : fabs(kl + e.L);
    out[2] = fault ? inf : inv_tau * (e.shkl + e.L);
    out[3] = fault ? inf : inv_tau * e.shkl;
    // a_n = (-1)^(n-1) / (n(n+1)) sum f^neq^(n+1) / f^n
    R dev = R(0);
    if (e.a1 != R(0)) {
        const R ia1 = rcp(R(0.5) * e.a1);
        const R r2 = R(-1.0 / 6.0) * e.a2 * ia1, r3 = R(1.0 / 12.0) * e.a3 * ia1,
                r4 = R(-1.0 / 20.0) * e.a4 * ia1;
        dev = R(4) * r2 - R(16) * r2 * r2 + R(8) * r3 - R(80) * r2 * r3 + R(80) * r2 * r2 * r2 + R(16) * r4;
    }
    out[4] = fault ? inf : fabs(dev);
    const R dxy = pxx - pyy;
    out[5] = inv_mu * sqrt(R(0.5) * dxy * dxy + R(2) * pxy * pxy);
    const R hx = ux * pxx + uy * pxy, hy = ux * pxy + uy * pyy;
    out[6] = sqrt(hx * hx + hy * hy);
    if (d2q25) {
        const R fx = qx - hx, fy = qy - hy;
        out[7] = sqrt(fx * fx + fy * fy);
        out[8] = R(0);
        out[9] = R(0);
    } else {
        out[7] = R(0);
        out[8] = R(0.70710678118654752) * fabs(pxx + pyy) * inv_mu;      // sqrt(2) |tr P| / (2 mu)
        out[9] = R(0.5) * inv_mu * sqrt(pxx * pxx + R(2) * pxy * pxy + pyy * pyy);
    }
}

// ---------------------------------------------------------------------------
// Explicit waits for kernels that stage through LDS with direct global->LDS
// loads.  The compiler does not reliably order LDS reads after such loads, so
// the kernels wait themselves; the empty asm statements keep the compiler from
// moving memory accesses across the wait.  s_waitcnt immediates (gfx9
// encoding): vmcnt in bits 3:0 and 15:14, expcnt in 6:4, lgkmcnt in 11:8.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wait_vmem_all()        // vmcnt(0)
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0x0F70);
    asm volatile("" ::: "memory");
}
__device__ __forceinline__ void wait_lds_all()         // lgkmcnt(0)
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xC07F);
    asm volatile("" ::: "memory");
}

// ---------------------------------------------------------------------------
// Reductions: wave64 butterfly in FP64, then across the 4 waves via LDS.
// Deterministic for a fixed launch shape.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Reduces acc[kNsums] over the block; thread 0 writes out[0..kNsums).
__device__ __forceinline__ void block_sums(double (&acc)[kNsums], double* __restrict__ out)
{
    __shared__ double red[kBlock / kWave][kNsums];
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
        for (int w = 0; w < kBlock / kWave; ++w) s += red[w][threadIdx.x];
        out[threadIdx.x] = s;
    }
}

} // namespace lks
