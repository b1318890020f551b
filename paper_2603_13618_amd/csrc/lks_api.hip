// lks_api.hip -- the extern "C" surface of liblks.so (declared in
// include/lks.h): validation, launch shapes, ping-pong bookkeeping, stream
// handling and error reporting.  All device memory belongs to the caller.
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "lks.h"
#include "lks_internal.h"

namespace {

constexpr int kBlock = 256;
constexpr int kMaxChunk = 64;          // steps whose partial sums are reduced together
constexpr size_t kHeader = 256;        // scratch: fault counter, padded
constexpr size_t kErrLen = 512;        // bytes of an error message, NUL included

// message of the last failed call that had no context (lks_create,
// lks_step_noalloc, lks_copy_probe), per host thread
thread_local char g_err[kErrLen];

int q_of(int lattice) { return lattice == LKS_D2Q9 ? 9 : (lattice == LKS_D2Q25 ? 25 : 0); }
int nsens_of(int lattice) { return lattice == LKS_D2Q9 ? 3 : (lattice == LKS_D2Q25 ? 4 : 0); }
bool ddf(const lks_config& c) { return c.model == LKS_MODEL_DDF; }
// stored planes of the state and base sensor planes of a configuration
int state_planes(const lks_config& c) { return ddf(c) ? 50 : q_of(c.lattice); }
int base_planes(const lks_config& c) { return ddf(c) ? 5 : nsens_of(c.lattice); }
double cv_of(const lks_config& c) { return 1.0 / (c.gamma - 1.0); }

// extension sensors: planes after the base planes, in increasing bit order
lks::ExtArgs ext_args(const lks_config& c)
{
    lks::ExtArgs x;
    x.mask = c.ext_mask;
    int p = base_planes(c);
    for (int k = 0; k < lks::kNumExtHost; ++k) {
        x.plane[k] = (c.ext_mask & (1u << k)) ? p++ : -1;
        for (int j = 0; j < 2; ++j) {
            x.thr[k][j] = c.thr_ext[k][j];
            x.thr_f[k][j] = (float)c.thr_ext[k][j];
        }
    }
    return x;
}

// Thresholds the kernels compare the base sensors with: those of the sensors
// in flag_mask, +INF for the others (a sensor compares false with +INF, NaN
// included), so the kernels take every base sensor without a branch on the
// mask.  The quasi-equilibrium sensor of the double distribution likewise.
double flag_thr(const lks_config& c, int s, int j)
{
    return (c.flag_mask & (1u << s)) ? c.thr[s][j] : INFINITY;
}
double flag_thr_qe(const lks_config& c, int j)
{
    return (c.flag_mask & LKS_S_QE) ? c.thr_qe[j] : INFINITY;
}

int planes_of(const lks_config& c) { return base_planes(c) + __builtin_popcount(c.ext_mask); }
size_t store_bytes(int dtype) { return dtype == LKS_F64 ? 8 : (dtype == LKS_F32 ? 4 : 2); }
size_t sens_bytes(int dtype) { return dtype == LKS_F64 ? 8 : 4; }
// cells per thread of the D2Q9 cell kernels when the hint is 0: FP32 four
// (16-byte accesses); FP64 two; 16-bit storage two, which leaves the kernel
// room for three waves per SIMD instead of two (BF16 / FP16 at 8192^2:
// 684 / 690 us per step against 705 / 716 with four cells)
int wide_vec(int dtype) { return dtype == LKS_F32 ? 4 : 2; }

// Launch shape of the D2Q9 cell kernels for a given vector width.
lks::GridShape d2q9_shape(const lks_config& c, int vec)
{
    lks::GridShape g;
    g.vec = vec;
    g.tiles_x = (c.nx + kBlock * vec - 1) / (kBlock * vec);
    int rows = c.launch_rows;
    if (rows <= 0 && c.layout == LKS_LAYOUT_ROWS && store_bytes(c.dtype) >= 4) {
        // row-interleaved FP32/FP64 state: two-row sweeps keep the workgroups
        // in flight on a narrow band of grid rows, i.e. on a few contiguous
        // stretches of HBM (FP32 at 4096^2 and 8192^2: 1 row 4-5 % slower,
        // 4 rows 6 %, 16 rows 14-20 %).  16-bit storage spends relatively
        // more time computing and keeps the long sweeps below.
        rows = 2;
    } else if (rows <= 0) {
        // at least ~1024 workgroups (4 per CU) with row sweeps of at most 16
        // rows: long enough to keep the next row in flight behind the
        // arithmetic, short enough to balance the CUs
        const long long target = 1024;
        long long r = ((long long)g.tiles_x * c.ny) / target;
        rows = (int)(r < 1 ? 1 : (r > 16 ? 16 : r));
    }
    if (rows > c.ny) rows = c.ny;
    g.rows = rows;
    const long long groups = (long long)((c.ny + rows - 1) / rows) * g.tiles_x;
    g.nblocks = (int)groups;
    return g;
}

const char* validate_config(const lks_config* c)
{
    if (!c) return "config is NULL";
    if (c->lattice != LKS_D2Q9 && c->lattice != LKS_D2Q25) return "lattice must be 9 or 25";
    if (c->nx < 1 || c->ny < 1) return "nx and ny must be >= 1";
    if ((long long)c->nx * c->ny > (1LL << 36)) return "grid too large";
    if (c->dtype < LKS_F64 || c->dtype > LKS_F16) return "dtype must be F64, F32, BF16 or F16";
    if (!(c->rho0 > 0.0) || !std::isfinite(c->rho0)) return "rho0 must be finite and > 0";
    if (c->max_steps < 1) return "max_steps must be >= 1";
    if (c->launch_rows < 0) return "launch_rows must be >= 0";
    if (c->launch_vec != 0 && c->launch_vec != 1 && c->launch_vec != 2 && c->launch_vec != 4)
        return "launch_vec must be 0, 1, 2 or 4";
    if (c->dtype == LKS_F64 && c->launch_vec == 4) return "launch_vec 4 is not available for F64";
    if (c->ext_reserved != 0) return "ext_reserved must be 0";
    const unsigned all_ext = (1u << LKS_MAX_EXT) - 1u;
    // QF needs the energy flux D2Q9 lacks; COMP and STRAIN divide by the
    // bulk viscosity, zero for the monatomic D2Q25 BGK gas
    const unsigned valid_ext = c->lattice == LKS_D2Q9 ? all_ext & ~(unsigned)LKS_X_QF
                             : c->model == LKS_MODEL_DDF ? all_ext
                                                          : all_ext & ~(unsigned)(LKS_X_COMP | LKS_X_STRAIN);
    if (c->ext_mask & ~valid_ext) return "ext_mask names a sensor this lattice does not have";
    if (c->model != LKS_MODEL_BGK && c->model != LKS_MODEL_DDF) return "model must be BGK or DDF";
    if (c->layout != LKS_LAYOUT_PLANES && c->layout != LKS_LAYOUT_ROWS) return "layout must be PLANES or ROWS";
    if (c->launch_nt < 0 || c->launch_nt > 2) return "launch_nt must be 0, 1 or 2";
    if (c->launch_steps < 0 || c->launch_steps > 2) return "launch_steps must be 0, 1 or 2";
    if (c->launch_steps == 2 && (c->lattice != LKS_D2Q9 || c->ext_mask))
        return "launch_steps 2 needs D2Q9 without extension sensors";
    if (c->model == LKS_MODEL_DDF) {
        if (c->lattice != LKS_D2Q25) return "the double distribution needs D2Q25";
        if (!(c->gamma > 1.0 && c->gamma < 2.0)) return "gamma must be in (1, 2)";
        if (!(c->prandtl > 0.0 && c->prandtl <= 1.0)) return "prandtl must be in (0, 1]";
        if (std::isnan(c->thr_qe[0]) || std::isnan(c->thr_qe[1])) return "threshold is NaN";
        if (c->thr_qe[0] > c->thr_qe[1]) return "thresholds must satisfy theta1 <= theta2";
    }
    const unsigned base = c->lattice == LKS_D2Q9 ? 7u : (c->model == LKS_MODEL_DDF ? 31u : 15u);
    const unsigned valid = base | (c->ext_mask << 8);
    if (c->flag_mask & ~valid) return "flag_mask names a sensor this configuration does not compute";
    for (int s = 0; s < LKS_MAX_SENSORS; ++s) {
        if (std::isnan(c->thr[s][0]) || std::isnan(c->thr[s][1])) return "threshold is NaN";
        if (c->thr[s][0] > c->thr[s][1]) return "thresholds must satisfy theta1 <= theta2";
    }
    for (int k = 0; k < LKS_MAX_EXT; ++k) {
        if (!(c->ext_mask & (1u << k))) continue;
        if (std::isnan(c->thr_ext[k][0]) || std::isnan(c->thr_ext[k][1])) return "threshold is NaN";
        if (c->thr_ext[k][0] > c->thr_ext[k][1]) return "thresholds must satisfy theta1 <= theta2";
    }
    if (c->lattice == LKS_D2Q9) {
        if (c->bc_x != LKS_PERIODIC || c->bc_y != LKS_PERIODIC) return "D2Q9 grids are periodic";
        if (!(c->tau > 0.5) || !std::isfinite(c->tau)) return "tau must be finite and > 0.5";
    } else {
        if ((c->bc_x != LKS_PERIODIC && c->bc_x != LKS_OUTFLOW) ||
            (c->bc_y != LKS_PERIODIC && c->bc_y != LKS_OUTFLOW))
            return "bc must be PERIODIC or OUTFLOW";
        if (!(c->mu > 0.0) || !(c->dt > 0.0) || !(c->dx > 0.0) || !std::isfinite(c->mu) ||
            !std::isfinite(c->dt) || !std::isfinite(c->dx))
            return "mu, dt and dx must be finite and > 0";
    }
    return nullptr;
}

lks::D2Q25Args d2q25_args(const lks_config& c)
{
    lks::D2Q25Args a;
    a.nx = c.nx;
    a.ny = c.ny;
    a.plane = (long long)c.nx * c.ny;
    a.L = lks::pop_layout(c.layout, state_planes(c), c.nx, c.ny);
    a.bc_x = c.bc_x;
    a.bc_y = c.bc_y;
    a.mu = c.mu;
    a.dt = c.dt;
    a.dx = c.dx;
    a.rho0 = c.rho0;
    for (int s = 0; s < LKS_MAX_SENSORS; ++s)
        for (int j = 0; j < 2; ++j) a.thr[s][j] = flag_thr(c, s, j);
    a.mask = c.flag_mask;
    a.x = ext_args(c);
    a.model = c.model;
    a.cv = ddf(c) ? cv_of(c) : 0.0;
    a.prandtl = ddf(c) ? c.prandtl : 1.0;
    a.thr_qe[0] = ddf(c) ? flag_thr_qe(c, 0) : INFINITY;
    a.thr_qe[1] = ddf(c) ? flag_thr_qe(c, 1) : INFINITY;
    a.aux = nullptr;
    a.nt_stores = 0;
    lks::d2q25_tile_shape(c.dtype, c.model, &a.tile_x, &a.tile_y);
    a.tiles_x = (c.nx + a.tile_x - 1) / a.tile_x;
    a.tiles_y = (c.ny + a.tile_y - 1) / a.tile_y;
    a.nblocks = a.tiles_x * a.tiles_y;
    return a;
}

// workgroups of one step's cell kernel: the most any vector width that
// lks_create may pick uses (the automatic sweep length grows with the tile
// count, so the narrowest vector does not always have the most workgroups)
int step_blocks(const lks_config& c)
{
    if (c.lattice == LKS_D2Q25) return d2q25_args(c).nblocks;
    int nb = c.launch_steps == 2 ? lks::d2q9_two_blocks(c.dtype, c.nx, c.ny) : 0;
    for (int vec : {1, 2, 4}) {
        const int b = d2q9_shape(c, vec).nblocks;
        nb = b > nb ? b : nb;
    }
    return nb;
}

// steps whose partial sums share the scratch before one reduction launch
int chunk_steps(const lks_config& c)
{
    const long long per_step = (long long)step_blocks(c) * lks::kNsumsHost * sizeof(double);
    long long k = (16LL << 20) / (per_step > 0 ? per_step : 1);
    if (k < 1) k = 1;
    if (k > kMaxChunk) k = kMaxChunk;
    if (k > c.max_steps) k = c.max_steps;
    return (int)k;
}

size_t partials_bytes(const lks_config& c)
{
    const size_t b = (size_t)chunk_steps(c) * (size_t)step_blocks(c) * lks::kNsumsHost * sizeof(double);
    return (b + 255) / 256 * 256;
}

// the double distribution's per-cell hand-over between its two kernels
size_t aux_bytes(const lks_config& c)
{
    if (!ddf(c)) return 0;
    const size_t real = c.dtype == LKS_F64 ? 8 : 4;
    return (size_t)lks::kDdfAux * (size_t)c.nx * (size_t)c.ny * real;
}

size_t scratch_for(const lks_config& c) { return kHeader + partials_bytes(c) + aux_bytes(c); }

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

} // namespace

lks::PopLayout lks::pop_layout(int layout, int q, int nx, int ny)
{
    PopLayout L;
    L.nx = nx;
    L.pp = layout == LKS_LAYOUT_ROWS ? (long long)nx : (long long)nx * ny;
    L.pr = layout == LKS_LAYOUT_ROWS ? (long long)q * nx : (long long)nx;
    return L;
}

struct lks_ctx {
    lks_config cfg;
    lks_buffers buf;
    hipStream_t stream;
    int Q, nsens;
    long long n;
    int cur;
    int64_t steps;
    bool ready;
    int chunk;
    lks::D2Q9Args a9;
    lks::D2Q25Args a25;
    int nblocks;
    int nblocks2;          // workgroups of the two-step launches (launch_steps 2), else 0
    double* partials;
    unsigned long long* faults;
    char err[kErrLen];     // fixed storage: reporting an error allocates nothing
};

namespace {

// printf-style message into the context (or the thread's context-free slot)
__attribute__((format(printf, 3, 4))) lks_status fail(lks_ctx* c, lks_status s, const char* fmt, ...)
{
    char* dst = c ? c->err : g_err;
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(dst, kErrLen, fmt, ap);
    va_end(ap);
    return s;
}

lks_status hip_check(lks_ctx* c, hipError_t e, const char* what)
{
    if (e == hipSuccess) return LKS_OK;
    return fail(c, LKS_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// Checks shared by lks_create and lks_step_noalloc (the caller's scratch
// buffer is checked by lks_create only).
lks_status check_create(const lks_config* cfg, const lks_buffers* buf, bool need_scratch)
{
    if (const char* m = validate_config(cfg)) return fail(nullptr, LKS_EINVAL, "%s", m);
    if (!buf) return fail(nullptr, LKS_EINVAL, "buffers are NULL");
    if (cfg->lattice == LKS_D2Q25 && cfg->dtype != LKS_F32 && cfg->dtype != LKS_F64)
        return fail(nullptr, LKS_EUNSUPPORTED, "D2Q25 supports F32 and F64 storage");
    if (cfg->ext_mask && cfg->dtype != LKS_F32 && cfg->dtype != LKS_F64)
        return fail(nullptr, LKS_EUNSUPPORTED, "extension sensors need F32 or F64 storage");
    if (!buf->pop[0] || !buf->pop[1] || !buf->sensors || !buf->flags || !buf->sums ||
        (need_scratch && !buf->scratch))
        return fail(nullptr, LKS_EINVAL, "a buffer pointer is NULL");
    if (buf->pop[0] == buf->pop[1]) return fail(nullptr, LKS_EINVAL, "pop[0] and pop[1] alias");
    if (!aligned(buf->sums, 8)) return fail(nullptr, LKS_EINVAL, "sums must be 8-byte aligned");
    const size_t sb = store_bytes(cfg->dtype);
    if (!aligned(buf->pop[0], sb) || !aligned(buf->pop[1], sb) ||
        !aligned(buf->sensors, sens_bytes(cfg->dtype)))
        return fail(nullptr, LKS_EINVAL, "population or sensor buffer misaligned for its dtype");
    return LKS_OK;
}

// Fill a context for a validated configuration.  scratch: device memory of
// kHeader + `partials` + aux_bytes(cfg) bytes (fault counter, per-workgroup
// partial sums of as many steps as `partials` bytes hold, up to kMaxChunk,
// then the double distribution's hand-over).
void setup_ctx(lks_ctx* c, const lks_config& cfg, const lks_buffers& buf, hipStream_t stream, char* scratch,
               size_t partials)
{
    c->cfg = cfg;
    c->buf = buf;
    c->buf.scratch = scratch;
    c->stream = stream;
    c->Q = state_planes(cfg);
    c->nsens = planes_of(cfg);
    c->n = (long long)cfg.nx * cfg.ny;
    c->cur = 0;
    c->steps = 0;
    c->ready = false;
    c->faults = reinterpret_cast<unsigned long long*>(scratch);
    c->partials = reinterpret_cast<double*>(scratch + kHeader);
    void* aux = aux_bytes(cfg) ? scratch + kHeader + partials : nullptr;

    // widest vector the row length and buffer alignment allow (or the hint)
    const size_t sb = store_bytes(cfg.dtype);
    int vec = cfg.launch_vec > 0 ? cfg.launch_vec : wide_vec(cfg.dtype);
    const size_t vbytes = sb * vec;
    if (cfg.nx % vec != 0 || !aligned(buf.pop[0], vbytes) || !aligned(buf.pop[1], vbytes) ||
        !aligned(buf.sensors, sens_bytes(cfg.dtype) * vec) || !aligned(buf.flags, vec))
        vec = 1;
    lks::D2Q9Args& a = c->a9;
    a.nx = cfg.nx;
    a.ny = cfg.ny;
    a.plane = c->n;
    a.L = lks::pop_layout(cfg.layout, c->Q, cfg.nx, cfg.ny);
    a.tau = cfg.tau;
    a.rho0 = cfg.rho0;
    a.mask = cfg.flag_mask;
    a.g = d2q9_shape(cfg, vec);
    a.inv_tau_f = (float)(1.0 / cfg.tau);
    a.rho0_f = (float)cfg.rho0;
    for (int s = 0; s < LKS_MAX_SENSORS; ++s) {
        for (int k = 0; k < 2; ++k) {
            a.thr[s][k] = flag_thr(cfg, s, k);
            a.thr_f[s][k] = (float)a.thr[s][k];
        }
    }
    a.x = ext_args(cfg);
    // Non-temporal stores in the fused D2Q9 step when the two state buffers
    // exceed the 256 MB last-level cache: the next step's loads then come
    // from HBM either way and the hint keeps the stores from evicting the
    // rows still to be read (FP32: 2048^2 4 %, 4096^2 7 %, 8192^2 8 % faster,
    // FP64 4096^2 5 %).  Below that size the states stay cache-resident
    // between steps, and the hint costs (BF16 2048^2 10 %, the 1024^2
    // adjoint 9 %).
    a.nt_stores = cfg.launch_nt == 2 ? 1
                : cfg.launch_nt == 1 ? 0
                : (2.0 * c->Q * (double)c->n * (double)sb > 256.0 * (1 << 20) ? 1 : 0);
    c->a25 = d2q25_args(cfg);
    c->a25.aux = aux;
    c->a25.nt_stores = a.nt_stores;
    c->nblocks = cfg.lattice == LKS_D2Q25 ? c->a25.nblocks : a.g.nblocks;
    c->nblocks2 = cfg.launch_steps == 2 ? lks::d2q9_two_blocks(cfg.dtype, cfg.nx, cfg.ny) : 0;
    // as many steps per reduction launch as the partials area holds for the
    // launch with the most workgroups
    const int nbmax = c->nblocks2 > c->nblocks ? c->nblocks2 : c->nblocks;
    const long long per_step = (long long)nbmax * lks::kNsumsHost * (long long)sizeof(double);
    long long k = (long long)partials / per_step;
    if (k > kMaxChunk) k = kMaxChunk;
    if (k > cfg.max_steps) k = cfg.max_steps;
    // two steps per launch pair the steps of one reduction batch: an even
    // batch pairs all of them, and only the odd last step of a call runs
    // alone (in the one-step kernel)
    if (cfg.launch_steps == 2 && k > 1) k &= ~1LL;
    c->chunk = (int)(k < 1 ? 1 : k);
}

// The step loop of lks_step and lks_step_noalloc (c valid).
lks_status step_impl(lks_ctx* c, int32_t nsteps, int32_t fused)
{
    if (nsteps < 0) return fail(c, LKS_EINVAL, "nsteps must be >= 0");
    if (fused != 0 && fused != 1) return fail(c, LKS_EINVAL, "fused must be 0 or 1");
    if (!c->ready) return fail(c, LKS_ESTATE, "step before init_equilibrium or restore");
    const bool q25 = c->cfg.lattice == LKS_D2Q25;
    if (q25 && !fused) return fail(c, LKS_EUNSUPPORTED, "the unfused passes exist for D2Q9 only");
    if (c->cfg.ext_mask && !fused)
        return fail(c, LKS_EUNSUPPORTED, "extension sensors are computed by the fused step only");
    const lks::D2Q9Args& a = c->a9;
    int done = 0;
    while (done < nsteps) {
        int m = (nsteps - done) < c->chunk ? (nsteps - done) : c->chunk;
        // two steps per launch: the batch takes whole pairs; a step without a
        // partner (the odd end of a call, or batches of one) is a batch of
        // its own in the one-step kernel
        const bool two = fused && c->nblocks2 > 0 && m >= 2;
        if (two) m &= ~1;
        const int nb = two ? c->nblocks2 : c->nblocks;
        for (int s = 0; two && s < m; s += 2) {
            double* pa = c->partials + (size_t)s * nb * lks::kNsumsHost;
            hipError_t e = lks::launch_d2q9_two(c->cfg.dtype, a, c->buf.pop[c->cur], c->buf.pop[1 - c->cur],
                                                c->buf.sensors, c->buf.flags, pa,
                                                pa + (size_t)nb * lks::kNsumsHost, c->faults, c->stream);
            if (lks_status st = hip_check(c, e, "step kernel")) return st;
            c->cur = 1 - c->cur;
        }
        for (int s = 0; !two && s < m; ++s) {
            double* part = c->partials + (size_t)s * nb * lks::kNsumsHost;
            void* f = c->buf.pop[c->cur];
            void* g = c->buf.pop[1 - c->cur];
            hipError_t e;
            if (q25) {
                e = lks::launch_d2q25(c->cfg.dtype, c->a25, f, g, c->buf.sensors, c->buf.flags, part,
                                      c->faults, c->stream);
                if (e == hipSuccess) c->cur = 1 - c->cur;
            } else if (fused) {
                e = lks::launch_d2q9(c->cfg.dtype, lks::kFused, a, f, g, c->buf.sensors,
                                     c->buf.flags, part, c->faults, c->stream);
                if (e == hipSuccess) c->cur = 1 - c->cur;
            } else {
                e = lks::launch_d2q9(c->cfg.dtype, lks::kStream, a, f, g, nullptr, nullptr,
                                     nullptr, nullptr, c->stream);
                if (e == hipSuccess)
                    e = lks::launch_d2q9(c->cfg.dtype, lks::kSense, a, g, nullptr, c->buf.sensors,
                                         c->buf.flags, part, c->faults, c->stream);
                if (e == hipSuccess)
                    e = lks::launch_d2q9(c->cfg.dtype, lks::kCollide, a, g, f, nullptr, nullptr,
                                         nullptr, nullptr, c->stream);
            }
            if (lks_status st = hip_check(c, e, "step kernel")) return st;
        }
        const double mass_ref = (double)c->n * c->cfg.rho0;
        // sum_i w_i |v_i|^2 / 2 = 1 on D2Q25; the double distribution adds
        // (C_v - 1) rho0 of g per cell
        const double energy_ref = !q25 ? 0.0 : (ddf(c->cfg) ? cv_of(c->cfg) * mass_ref : mass_ref);
        hipError_t e = lks::launch_finalize(c->partials, nb, m, c->buf.sums, c->steps,
                                            c->cfg.max_steps, mass_ref, energy_ref, c->stream);
        if (lks_status st = hip_check(c, e, "finalize kernel")) return st;
        c->steps += m;
        done += m;
    }
    return LKS_OK;
}


constexpr int kMaxDevices = 64;

} // namespace

// Device scratch of lks_step_noalloc: the fault counter, the per-workgroup
// FP64 partial sums and, for the double distribution, the per-cell hand-over.
// One copy per GPU, held until the process ends.  In host code this name is
// only a handle for hipGetSymbolAddress: kernels and copies take the device
// address that call returns.
static __device__ __align__(256) unsigned char scratch[LKS_NOALLOC_SCRATCH_BYTES];

namespace {

// the address of `scratch` on each device, looked up once per device with
// that device current
std::atomic<void*> g_scratch_dev[kMaxDevices];
std::mutex g_scratch_mu;

lks_status noalloc_scratch(void** out)
{
    int dev = -1;
    if (lks_status s = hip_check(nullptr, hipGetDevice(&dev), "hipGetDevice")) return s;
    if (dev < 0 || dev >= kMaxDevices) return fail(nullptr, LKS_EUNSUPPORTED, "device index %d out of range", dev);
    void* p = g_scratch_dev[dev].load(std::memory_order_acquire);
    if (!p) {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        p = g_scratch_dev[dev].load(std::memory_order_relaxed);
        if (!p) {
            if (lks_status s = hip_check(nullptr, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)),
                                         "hipGetSymbolAddress(scratch)"))
                return s;
            if (!p) return fail(nullptr, LKS_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
            g_scratch_dev[dev].store(p, std::memory_order_release);
        }
    }
    *out = p;
    return LKS_OK;
}

} // namespace

extern "C" {

size_t lks_scratch_bytes(const lks_config* cfg)
{
    if (validate_config(cfg)) return 0;
    return scratch_for(*cfg);
}

int32_t lks_num_sensors(int32_t lattice) { return nsens_of(lattice); }

int32_t lks_sensor_planes(const lks_config* cfg)
{
    if (validate_config(cfg)) return 0;
    return planes_of(*cfg);
}

lks_status lks_create(const lks_config* cfg, const lks_buffers* buf, void* hip_stream, lks_ctx** out)
{
    if (!out) return fail(nullptr, LKS_EINVAL, "out is NULL");
    *out = nullptr;
    if (lks_status st = check_create(cfg, buf, true)) return st;
    const size_t need = scratch_for(*cfg);
    if (buf->scratch_bytes < need) return fail(nullptr, LKS_EINVAL, "scratch too small: need %zu bytes", need);
    if (!aligned(buf->scratch, 8)) return fail(nullptr, LKS_EINVAL, "scratch must be 8-byte aligned");
    lks_ctx* c = new (std::nothrow) lks_ctx();
    if (!c) return fail(nullptr, LKS_EINVAL, "out of host memory");
    setup_ctx(c, *cfg, *buf, static_cast<hipStream_t>(hip_stream), static_cast<char*>(buf->scratch),
              partials_bytes(*cfg));
    *out = c;
    return LKS_OK;
}

lks_status lks_init_equilibrium(lks_ctx* c, const double* rho, const double* ux, const double* uy,
                                const double* T)
{
    if (!c) return LKS_EINVAL;
    if (!rho || !ux || !uy) return fail(c, LKS_EINVAL, "rho, ux and uy are required");
    if (c->cfg.lattice == LKS_D2Q25 && !T) return fail(c, LKS_EINVAL, "T is required on D2Q25");
    hipError_t e = ddf(c->cfg)
                       ? lks::launch_d2q25_ddf_init(c->cfg.dtype, c->n, c->a25.L, c->cfg.rho0, cv_of(c->cfg),
                                                    rho, ux, uy, T, c->buf.pop[0], c->stream)
                   : c->cfg.lattice == LKS_D2Q25
                       ? lks::launch_d2q25_init(c->cfg.dtype, c->n, c->a25.L, c->cfg.rho0, rho, ux, uy, T,
                                                c->buf.pop[0], c->stream)
                       : lks::launch_d2q9_init(c->cfg.dtype, c->n, c->a9.L, c->cfg.rho0, rho, ux, uy,
                                               c->buf.pop[0], c->stream);
    if (lks_status s = hip_check(c, e, "init kernel")) return s;
    if (lks_status s = hip_check(c, lks::launch_zero(c->faults, 1, c->stream), "zero kernel")) return s;
    c->cur = 0;
    c->steps = 0;
    c->ready = true;
    return LKS_OK;
}

lks_status lks_restore(lks_ctx* c, int32_t pop_index, int64_t steps_done)
{
    if (!c) return LKS_EINVAL;
    if (pop_index != 0 && pop_index != 1) return fail(c, LKS_EINVAL, "pop_index must be 0 or 1");
    if (steps_done < 0) return fail(c, LKS_EINVAL, "steps_done must be >= 0");
    if (lks_status s = hip_check(c, lks::launch_zero(c->faults, 1, c->stream), "zero kernel")) return s;
    c->cur = pop_index;
    c->steps = steps_done;
    c->ready = true;
    return LKS_OK;
}

lks_status lks_step(lks_ctx* c, int32_t nsteps, int32_t fused)
{
    if (!c) return LKS_EINVAL;
    return step_impl(c, nsteps, fused);
}

lks_status lks_step_noalloc(const lks_config* cfg, const lks_buffers* buf, void* hip_stream, int32_t pop_index,
                            int64_t steps_done, int32_t nsteps, int32_t fused, int32_t* pop_index_out)
{
    if (!pop_index_out) return fail(nullptr, LKS_EINVAL, "pop_index_out is NULL");
    if (lks_status st = check_create(cfg, buf, false)) return st;
    if (buf->scratch || buf->scratch_bytes)
        return fail(nullptr, LKS_EINVAL, "scratch must be NULL and scratch_bytes 0 (the library's array is used)");
    if (pop_index != 0 && pop_index != 1) return fail(nullptr, LKS_EINVAL, "pop_index must be 0 or 1");
    if (steps_done < 0) return fail(nullptr, LKS_EINVAL, "steps_done must be >= 0");
    if (nsteps < 0) return fail(nullptr, LKS_EINVAL, "nsteps must be >= 0");
    if (fused != 0 && fused != 1) return fail(nullptr, LKS_EINVAL, "fused must be 0 or 1");
    // the partial sums of at least one step, behind the header, before the hand-over
    const size_t aux = aux_bytes(*cfg);
    const size_t room = (size_t)LKS_NOALLOC_SCRATCH_BYTES - kHeader;
    const size_t one = (size_t)step_blocks(*cfg) * lks::kNsumsHost * sizeof(double);
    if (aux > room || room - aux < one)
        return fail(nullptr, LKS_EINVAL, "configuration needs %zu bytes of scratch, more than the %u the "
                    "library holds per device", kHeader + one + aux, (unsigned)LKS_NOALLOC_SCRATCH_BYTES);
    const size_t partials = (room - aux) / 256 * 256;
    void* base = nullptr;
    if (lks_status st = noalloc_scratch(&base)) return st;

    lks_ctx c{};
    setup_ctx(&c, *cfg, *buf, static_cast<hipStream_t>(hip_stream), static_cast<char*>(base), partials);
    // as lks_restore: the state in pop[pop_index] after steps_done steps, faults cleared
    c.cur = pop_index;
    c.steps = steps_done;
    c.ready = true;
    lks_status st = hip_check(&c, lks::launch_zero(c.faults, 1, c.stream), "zero kernel");
    if (st == LKS_OK) st = step_impl(&c, nsteps, fused);
    if (st != LKS_OK) {
        std::memcpy(g_err, c.err, kErrLen);
        return st;
    }
    *pop_index_out = c.cur;
    return LKS_OK;
}

lks_status lks_current(const lks_ctx* c, int32_t* pop_index, int64_t* steps_done)
{
    if (!c) return LKS_EINVAL;
    if (pop_index) *pop_index = c->cur;
    if (steps_done) *steps_done = c->steps;
    return LKS_OK;
}

lks_status lks_moments(lks_ctx* c, double* rho, double* ux, double* uy, double* T)
{
    if (!c) return LKS_EINVAL;
    if (!rho || !ux || !uy) return fail(c, LKS_EINVAL, "rho, ux and uy are required");
    if (!c->ready) return fail(c, LKS_ESTATE, "moments before init_equilibrium or restore");
    hipError_t e = ddf(c->cfg)
                       ? lks::launch_d2q25_ddf_moments(c->cfg.dtype, c->n, c->a25.L, c->cfg.rho0,
                                                       cv_of(c->cfg), c->buf.pop[c->cur], rho, ux, uy, T,
                                                       c->stream)
                   : c->cfg.lattice == LKS_D2Q25
                       ? lks::launch_d2q25_moments(c->cfg.dtype, c->n, c->a25.L, c->cfg.rho0,
                                                   c->buf.pop[c->cur], rho, ux, uy, T, c->stream)
                       : lks::launch_d2q9_moments(c->cfg.dtype, c->n, c->a9.L, c->cfg.rho0,
                                                  c->buf.pop[c->cur], rho, ux, uy, T, c->stream);
    return hip_check(c, e, "moments kernel");
}

lks_status lks_read_host(lks_ctx* c, int32_t what, void* dst, size_t bytes)
{
    if (!c) return LKS_EINVAL;
    if (!dst) return fail(c, LKS_EINVAL, "host_dst is NULL");
    const void* src = nullptr;
    size_t size = 0;
    switch (what) {
    case 0: src = c->buf.pop[c->cur]; size = (size_t)c->Q * c->n * store_bytes(c->cfg.dtype); break;
    case 1: src = c->buf.sensors; size = (size_t)c->nsens * c->n * sens_bytes(c->cfg.dtype); break;
    case 2: src = c->buf.flags; size = (size_t)c->n; break;
    case 3: src = c->buf.sums; size = (size_t)c->cfg.max_steps * LKS_NSUMS * sizeof(double); break;
    default: return fail(c, LKS_EINVAL, "what must be 0..3");
    }
    if (bytes != size) return fail(c, LKS_EINVAL, "bytes must be %zu", size);
    if (lks_status s = hip_check(c, hipStreamSynchronize(c->stream), "stream sync")) return s;
    return hip_check(c, hipMemcpy(dst, src, size, hipMemcpyDeviceToHost), "copy to host");
}

lks_status lks_check(lks_ctx* c, int64_t* n_nonpos)
{
    if (!c) return LKS_EINVAL;
    if (lks_status s = hip_check(c, hipStreamSynchronize(c->stream), "stream sync")) return s;
    unsigned long long nf = 0;
    if (lks_status s = hip_check(c, hipMemcpy(&nf, c->faults, sizeof(nf), hipMemcpyDeviceToHost),
                                 "read fault counter"))
        return s;
    if (n_nonpos) *n_nonpos = (int64_t)nf;
    const long long rows = c->steps < c->cfg.max_steps ? c->steps : c->cfg.max_steps;
    if (rows > 0) {
        // in pieces through a small host buffer
        double h[64 * LKS_NSUMS];
        for (long long r0 = 0; r0 < rows; r0 += 64) {
            const long long nr = rows - r0 < 64 ? rows - r0 : 64;
            if (lks_status s = hip_check(c, hipMemcpy(h, c->buf.sums + r0 * LKS_NSUMS,
                                                      (size_t)nr * LKS_NSUMS * sizeof(double),
                                                      hipMemcpyDeviceToHost), "read sums"))
                return s;
            for (long long r = 0; r < nr; ++r)
                for (int k = 0; k < 3; ++k)
                    if (std::isnan(h[r * LKS_NSUMS + k]))
                        return fail(c, LKS_ENAN, "a mass or momentum sum is NaN");
        }
    }
    if (nf > 0) return fail(c, LKS_ENONPOS, "%llu positivity-fault cells", nf);
    return LKS_OK;
}

lks_status lks_macro_sensors(lks_ctx* c, const double* rho, const double* ux, const double* uy,
                             const double* T, const lks_transport* tr, uint32_t which, double* out)
{
    if (!c) return LKS_EINVAL;
    if (!tr) return fail(c, LKS_EINVAL, "transport is NULL");
    if (tr->reserved != 0) return fail(c, LKS_EINVAL, "transport reserved field must be 0");
    if (!std::isfinite(tr->mu) || !std::isfinite(tr->lambda) || !std::isfinite(tr->kappa))
        return fail(c, LKS_EINVAL, "transport coefficients must be finite");
    if (which == 0 || (which >> lks::kNumMacro) != 0) return fail(c, LKS_EINVAL, "which names no or unknown sensors");
    if (!ux || !uy || !out) return fail(c, LKS_EINVAL, "ux, uy and out are required");
    if ((which & (lks::kMacroQF | lks::kMacroQNSF)) && !T) return fail(c, LKS_EINVAL, "T is required for QF and QNSF");
    if (tr->per_rho && !rho) return fail(c, LKS_EINVAL, "rho is required with per_rho");
    if (out == ux || out == uy || out == T || out == rho) return fail(c, LKS_EINVAL, "out must not alias an input");
    const bool aligned8 = aligned(ux, 8) && aligned(uy, 8) && aligned(out, 8) && (!T || aligned(T, 8)) &&
                          (!rho || aligned(rho, 8));
    if (!aligned8) return fail(c, LKS_EINVAL, "fields must be 8-byte aligned");
    lks::MacroArgs a;
    a.nx = c->cfg.nx;
    a.ny = c->cfg.ny;
    a.bc_x = c->cfg.bc_x;
    a.bc_y = c->cfg.bc_y;
    a.plane = c->n;
    a.inv2dx = 0.5 / (c->cfg.lattice == LKS_D2Q9 ? 1.0 : c->cfg.dx);
    a.mu = tr->mu;
    a.lam = tr->lambda;
    a.kappa = tr->kappa;
    a.per_rho = tr->per_rho ? 1 : 0;
    a.which = which;
    int p = 0;
    for (int k = 0; k < lks::kNumMacro; ++k) a.plane_of[k] = (which & (1u << k)) ? p++ : -1;
    return hip_check(c, lks::launch_macro(a, rho, ux, uy, T, out, c->stream), "macro sensors");
}

lks_status lks_tag_buffer(lks_ctx* c, int32_t b, const uint8_t* flags, uint8_t* levels)
{
    if (!c) return LKS_EINVAL;
    if (!flags || !levels) return fail(c, LKS_EINVAL, "flags or levels is NULL");
    if (flags == levels) return fail(c, LKS_EINVAL, "flags and levels must not alias");
    if (b < 0 || b > lks::kMaxBuffer) return fail(c, LKS_EINVAL, "buffer width out of range");
    return hip_check(c, lks::launch_tag_buffer(flags, levels, c->cfg.nx, c->cfg.ny, c->cfg.bc_x,
                                                c->cfg.bc_y, b, c->stream),
                      "tag buffer");
}

lks_status lks_tag_tiles(lks_ctx* c, const uint8_t* levels, int32_t level, int32_t ts, int32_t* counts)
{
    if (!c) return LKS_EINVAL;
    if (!levels || !counts) return fail(c, LKS_EINVAL, "levels or counts is NULL");
    if (ts < 1 || ts > 64) return fail(c, LKS_EINVAL, "tile size must be 1 .. 64");
    if (level < 1 || level > 2) return fail(c, LKS_EINVAL, "level must be 1 or 2");
    if (!aligned(counts, 4)) return fail(c, LKS_EINVAL, "counts misaligned");
    return hip_check(c, lks::launch_tag_tiles(levels, counts, c->cfg.nx, c->cfg.ny, level, ts, c->stream),
                      "tag tiles");
}

lks_status lks_step_from(lks_ctx* c, const void* src, void* dst)
{
    if (!c) return LKS_EINVAL;
    if (!src || !dst) return fail(c, LKS_EINVAL, "src and dst are required");
    if (src == dst) return fail(c, LKS_EINVAL, "src and dst must differ");
    hipError_t e = c->cfg.lattice == LKS_D2Q25
                       ? lks::launch_d2q25(c->cfg.dtype, c->a25, src, dst, c->buf.sensors,
                                           c->buf.flags, c->partials, c->faults, c->stream)
                       : lks::launch_d2q9(c->cfg.dtype, lks::kFused, c->a9, src, dst,
                                          c->buf.sensors, c->buf.flags, c->partials, c->faults,
                                          c->stream);
    return hip_check(c, e, "step kernel");
}

namespace {
lks_status adjoint_ok(lks_ctx* c)
{
    if (c->cfg.lattice != LKS_D2Q9) return fail(c, LKS_EUNSUPPORTED, "the adjoint is D2Q9 only");
    if (c->cfg.dtype != LKS_F32 && c->cfg.dtype != LKS_F64)
        return fail(c, LKS_EUNSUPPORTED, "the adjoint needs F32 or F64 storage");
    return LKS_OK;
}
} // namespace

lks_status lks_adjoint_seed_kl(lks_ctx* c, const void* pop_prev, void* lam_out)
{
    if (!c) return LKS_EINVAL;
    if (lks_status s = adjoint_ok(c)) return s;
    if (!pop_prev || !lam_out) return fail(c, LKS_EINVAL, "pop_prev and lam_out are required");
    if (pop_prev == lam_out) return fail(c, LKS_EINVAL, "pop_prev and lam_out must differ");
    return hip_check(c, lks::launch_adj_seed(c->cfg.dtype, c->a9, pop_prev, lam_out, c->stream),
                     "adjoint seed kernel");
}

lks_status lks_adjoint_step(lks_ctx* c, const void* pop_prev, const void* lam_in, void* lam_out)
{
    if (!c) return LKS_EINVAL;
    if (lks_status s = adjoint_ok(c)) return s;
    if (!pop_prev || !lam_in || !lam_out)
        return fail(c, LKS_EINVAL, "pop_prev, lam_in and lam_out are required");
    if (lam_in == lam_out || pop_prev == lam_out)
        return fail(c, LKS_EINVAL, "lam_out must not alias an input");
    return hip_check(c, lks::launch_adj_step(c->cfg.dtype, c->a9, pop_prev, lam_in, lam_out,
                                             c->stream),
                     "adjoint step kernel");
}

lks_status lks_adjoint_init(lks_ctx* c, const double* rho0, const double* ux0, const double* uy0,
                            const void* lam0, double* gux, double* guy)
{
    if (!c) return LKS_EINVAL;
    if (lks_status s = adjoint_ok(c)) return s;
    if (!rho0 || !ux0 || !uy0 || !lam0 || !gux || !guy)
        return fail(c, LKS_EINVAL, "all arguments are required");
    return hip_check(c, lks::launch_adj_init(c->cfg.dtype, c->a9, rho0, ux0, uy0, lam0, gux, guy,
                                             c->stream),
                     "adjoint init kernel");
}

lks_status lks_destroy(lks_ctx* c)
{
    delete c;
    return LKS_OK;
}

const char* lks_status_str(lks_status s)
{
    switch (s) {
    case LKS_OK: return "ok";
    case LKS_EINVAL: return "invalid argument";
    case LKS_ESTATE: return "call out of order";
    case LKS_EHIP: return "HIP runtime error";
    case LKS_ENONPOS: return "non-positive populations";
    case LKS_ENAN: return "NaN in global sums";
    case LKS_EUNSUPPORTED: return "unsupported combination";
    }
    return "unknown status";
}

const char* lks_last_error(const lks_ctx* c) { return c ? c->err : g_err; }

lks_status lks_copy_probe(void* dst, const void* src, size_t bytes, void* hip_stream)
{
    if (!dst || !src || bytes % 16 != 0 || !aligned(dst, 16) || !aligned(src, 16))
        return fail(nullptr, LKS_EINVAL, "copy probe needs 16-byte aligned pointers and sizes");
    hipError_t e = lks::launch_copy_probe(dst, src, bytes, static_cast<hipStream_t>(hip_stream));
    return hip_check(nullptr, e, "copy kernel");
}

} // extern "C"
