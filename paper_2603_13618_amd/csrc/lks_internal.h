// lks_internal.h -- launch interface between the C-ABI layer (lks_api.hip)
// and the kernel translation units.  Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lks {

constexpr int kNsumsHost = 8;   // doubles per partial / per step (LKS_NSUMS)

// Launch shape of the cell kernels: each thread owns `vec` consecutive cells
// of a row, a 256-thread workgroup spans 256*vec cells of `rows` consecutive
// rows, and workgroup b covers x-tile (b % tiles_x) of row group (b / tiles_x).
struct GridShape {
    int vec;
    int tiles_x;
    int rows;
    int nblocks;
};

constexpr int kNumExtHost = 10;    // extension sensors (LKS_MAX_EXT)
constexpr int kExtFlagShift = 8;   // flag_mask bit of extension sensor k: 8 + k

// Extension sensors of a launch: which are computed, where they are stored,
// and the thresholds of those that drive the flags.
struct ExtArgs {
    unsigned mask;                   // 0 = none (the kernels without them run)
    int plane[kNumExtHost];          // sensor plane of sensor k, -1 = not stored
    double thr[kNumExtHost][2];
    float thr_f[kNumExtHost][2];     // the same rounded to FP32
};

// Where population i of cell (x, y) lives in a state buffer: element
// i * pp + y * pr + x.  Plane-major [Q][ny][nx]: pp = nx * ny, pr = nx;
// row-interleaved [ny][Q][nx]: pp = nx, pr = Q * nx.  Sensors, flags and
// fields are always plane-major.
struct PopLayout {
    int nx;
    long long pp, pr;
    __host__ __device__ long long at(int i, int y, int x) const { return i * pp + y * pr + x; }
    // population i of cell c = y * nx + x
    __host__ __device__ long long cell(int i, long long c) const
    {
        const long long y = c / nx;
        return i * pp + y * pr + (c - y * nx);
    }
};
PopLayout pop_layout(int layout, int q, int nx, int ny);

struct D2Q9Args {
    int nx, ny;
    long long plane;          // nx * ny (sensor planes)
    PopLayout L;              // population planes
    double tau;
    double rho0;
    double thr[4][2];         // flag thresholds, +INF for sensors not in mask
    unsigned mask;
    GridShape g;
    // the same parameters rounded to FP32 on the host, so FP32 kernels keep
    // them in scalar registers
    float inv_tau_f, rho0_f;
    float thr_f[4][2];
    ExtArgs x;
    int nt_stores;            // fused step: non-temporal stores (large states)
};

struct D2Q25Args {
    int nx, ny;
    long long plane;          // nx * ny (sensor planes, hand-over planes)
    PopLayout L;              // population planes
    int bc_x, bc_y;           // 0 periodic, 1 outflow
    double mu, dt, dx;
    double rho0;
    double thr[4][2];         // flag thresholds, +INF for sensors not in mask
    unsigned mask;
    int tile_x, tile_y;       // cells per workgroup tile
    int tiles_x, tiles_y;
    int nblocks;
    ExtArgs x;
    // double distribution (model 1): f and g, quasi-equilibrium collision
    int model;
    double cv;                // C_v = R/(gamma - 1)
    double prandtl;           // Pr = tau1/tau2 (<= 1)
    double thr_qe[2];         // flag thresholds of the quasi-equilibrium sensor (+INF if not in mask)
    // per-cell hand-over of the double distribution's f pass to its g pass:
    // [6][plane] of drho, ux, uy, T - 1, q_g (x, y) in the compute type
    void* aux;
    int nt_stores;            // non-temporal population stores (large states)
};
constexpr int kDdfAux = 6;

// D2Q9 passes: the fused step and the three passes of the unfused baseline
enum Pass { kFused = 0, kStream = 1, kSense = 2, kCollide = 3 };

// dtype: 0 f64, 1 f32, 2 bf16, 3 f16 (storage of the deviations)
hipError_t launch_d2q9(int dtype, int pass, const D2Q9Args& a, const void* fin, void* fout,
                       void* sens, uint8_t* flags, double* partials,
                       unsigned long long* faults, hipStream_t s);
// two fused D2Q9 steps per launch; the sums of the first step go to part_a,
// of the second to part_b
hipError_t launch_d2q9_two(int dtype, const D2Q9Args& a, const void* fin, void* fout, void* sens,
                           uint8_t* flags, double* part_a, double* part_b, unsigned long long* faults,
                           hipStream_t s);
// workgroups of one launch_d2q9_two launch
int d2q9_two_blocks(int dtype, int nx, int ny);

hipError_t launch_d2q25(int dtype, const D2Q25Args& a, const void* fin, void* fout, void* sens,
                        uint8_t* flags, double* partials, unsigned long long* faults,
                        hipStream_t s);
// workgroup tile (cells) of the D2Q25 kernel for a storage type and model
void d2q25_tile_shape(int dtype, int model, int* tx, int* ty);

// equilibrium initial states from FP64 fields [ny][nx] (n = nx*ny cells)
hipError_t launch_d2q9_init(int dtype, long long n, const PopLayout& L, double rho0, const double* rho,
                            const double* ux, const double* uy, void* pop, hipStream_t s);
hipError_t launch_d2q25_init(int dtype, long long n, const PopLayout& L, double rho0, const double* rho,
                             const double* ux, const double* uy, const double* T, void* pop,
                             hipStream_t s);

// FP64 moments of a stored state (T may be null)
hipError_t launch_d2q9_moments(int dtype, long long n, const PopLayout& L, double rho0, const void* pop,
                               double* rho, double* ux, double* uy, double* T, hipStream_t s);
hipError_t launch_d2q25_moments(int dtype, long long n, const PopLayout& L, double rho0, const void* pop,
                                double* rho, double* ux, double* uy, double* T, hipStream_t s);
// double distribution: 50 populations per cell (f deviations, then g
// deviations from (C_v - 1) w_i rho0)
hipError_t launch_d2q25_ddf_init(int dtype, long long n, const PopLayout& L, double rho0, double cv,
                                 const double* rho, const double* ux, const double* uy, const double* T,
                                 void* pop, hipStream_t s);
hipError_t launch_d2q25_ddf_moments(int dtype, long long n, const PopLayout& L, double rho0, double cv,
                                    const void* pop, double* rho, double* ux, double* uy, double* T,
                                    hipStream_t s);

// Reduce partials[step][nblocks][8] of nsteps steps into sums rows
// (row0 + step) mod max_rows; adds the reference mass/energy n_cells*rho0*(1, e_ref).
// The partials are scratch: chunk sums are written over them.
hipError_t launch_finalize(double* partials, int nblocks, int nsteps, double* sums,
                           long long row0, int max_rows, double mass_ref, double energy_ref,
                           hipStream_t s);

// adjoint kernels (D2Q9, F32/F64 storage)
hipError_t launch_adj_seed(int dtype, const D2Q9Args& a, const void* pop_prev, void* lam_out,
                           hipStream_t s);
hipError_t launch_adj_step(int dtype, const D2Q9Args& a, const void* pop_prev,
                           const void* lam_in, void* lam_out, hipStream_t s);
hipError_t launch_adj_init(int dtype, const D2Q9Args& a, const double* rho0,
                           const double* ux0, const double* uy0, const void* lam0,
                           double* gux, double* guy, hipStream_t s);

hipError_t launch_copy_probe(void* dst, const void* src, size_t bytes, hipStream_t s);

// regridding hand-off
constexpr int kMaxBuffer = 8;      // LKS_MAX_BUFFER
// macroscopic class-1 sensors (central differences)
constexpr int kNumMacro = 7;
constexpr unsigned kMacroQF = 1u << 5, kMacroQNSF = 1u << 6;
struct MacroArgs {
    int nx, ny, bc_x, bc_y;
    long long plane;
    double inv2dx, mu, lam, kappa;
    int per_rho;
    unsigned which;
    int plane_of[kNumMacro];
};
hipError_t launch_macro(const MacroArgs& a, const double* rho, const double* ux, const double* uy,
                        const double* T, double* out, hipStream_t s);

hipError_t launch_tag_buffer(const uint8_t* flags, uint8_t* out, int nx, int ny, int bc_x, int bc_y,
                             int b, hipStream_t s);
hipError_t launch_tag_tiles(const uint8_t* levels, int* counts, int nx, int ny, int level, int ts,
                            hipStream_t s);

// clears nwords 8-byte words with a fill kernel
hipError_t launch_zero(void* p, long long nwords, hipStream_t s);

} // namespace lks
