/*
 * lks.h -- C ABI of liblks.so: the fused kinetic update with local kinetic
 * refinement sensors on AMD Instinct MI355X (gfx950).
 *
 * Method ("Local kinetic sensors for adaptive mesh and algorithm refinement",
 * arXiv 2603.13618):
 *   - populations f_i on a tensor-product Gauss-Hermite velocity set
 *     (Sec. II.A.3): D2Q9 (GH3 x GH3, velocities in {-1,0,1}^2, T_ref = 1/3,
 *     isothermal, order-2 Grad-Hermite equilibrium) or D2Q25 (GH5 x GH5,
 *     T_ref = 1, order-4 Grad-Hermite equilibrium);
 *   - D2Q9: one lattice-BGK step = pull streaming g_i(x) = f_i(x - c_i) on a
 *     periodic grid, then f_i' = g_i - (g_i - f^eq_i)/tau (the collision of
 *     Sec. II.A.1 with tau1 = tau2);
 *   - D2Q25: one explicit-Euler finite-volume step (eq. finalDiscretePDE)
 *     with van Leer limited upwind fluxes and BGK relaxation, tau = mu/(rho T);
 *   - in the same pass, on the pre-collision populations of the step, the
 *     sensors S_KL (eq. HKL-sensor), S_NEQ (eq. sensor-neq-kin), S_PI
 *     (eq. sensor-TauNS-kin) and, on D2Q25, S_Q (eq. sensor-qNSF-kin-ryk,
 *     g = 0), and the per-cell refinement flag (Sec. II.B.2, regridding step 1);
 *   - optionally, in the same pass, the rest of Table I on the f distribution
 *     (the LKS_X_* extension sensors below).
 *
 * Conventions
 *   Layout: structure of arrays, x fastest.  Sensors, flags and fields are
 *     plane-major [k][ny][nx].  Populations follow the configured layout:
 *     LKS_LAYOUT_PLANES [Q][ny][nx] (f_i(x, y) at element (i*ny + y)*nx + x)
 *     or LKS_LAYOUT_ROWS [ny][Q][nx] (at (y*Q + i)*nx + x: the Q rows of one
 *     grid row lie together, so a step touches a few long runs of HBM
 *     instead of one run per population plane).  Both layouts hold the
 *     same values and every kernel gives bit-identical results on them.
 *     Population index i = q1*a + b, a = x-node, b = y-node index (ascending),
 *     q1 = 3 or 5.  D2Q9 velocity i is (a-1, b-1).
 *   Storage: populations are stored as deviations d_i = f_i - w_i*rho0 in the
 *     configured dtype (F64, F32, BF16, F16; 16-bit formats rounded to nearest
 *     even); all arithmetic is FP32 (FP64 for F64 storage); global sums are
 *     FP64.
 *   Sensors: plane s = 0 S_KL, 1 S_NEQ, 2 S_PI, 3 S_Q (D2Q25 only), so D2Q9
 *     has 3 base planes and D2Q25 4; then one plane per extension sensor in
 *     ext_mask, in increasing bit order (lks_sensor_planes counts them).
 *     float, or double for F64 storage.
 *   Flags: uint8 per cell; bits 0-1 = refinement level = max over the sensors
 *     enabled in flag_mask (base sensor s: bit s, thresholds thr[s]; extension
 *     sensor k: bit LKS_FLAG_X(k), thresholds thr_ext[k]) of
 *     [s > theta1] + [s > theta2]; bit 7 = positivity fault (some f_i or
 *     f^eq_i not > 0, or NaN: S_KL = +inf, level 2).
 *   Sums: per step LKS_NSUMS doubles: total mass, x- and y-momentum, total
 *     energy (0 on D2Q9), then the totals of S_KL, S_NEQ, S_PI, S_Q over all
 *     cells, all of the pre-collision state.  Step k (counted from 1 since
 *     init) writes row (k-1) mod max_steps.
 *
 * Ownership: the caller allocates and frees ALL device memory (buffers must
 *   outlive their use by the context); the context holds pointers, parameters
 *   and a few bytes of host state.  lks_destroy frees only the context.
 * Streams: every call that launches work enqueues it on the stream given at
 *   creation and returns without waiting; device errors surface at the next
 *   call that synchronises (lks_read_host, lks_check).  One context serves one
 *   stream and one host thread at a time.
 * Errors: every call returns an lks_status and throws nothing.  Invalid
 *   arguments return LKS_EINVAL before anything is launched; lks_last_error
 *   gives the message.
 */
#ifndef LKS_H
#define LKS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LKS_NSUMS 8
#define LKS_MAX_SENSORS 4

typedef struct lks_ctx lks_ctx;

typedef enum {
    LKS_OK = 0,
    LKS_EINVAL = 1,       /* invalid argument or configuration              */
    LKS_ESTATE = 2,       /* call out of order (e.g. step before init)      */
    LKS_EHIP = 3,         /* HIP runtime error (message in lks_last_error)  */
    LKS_ENONPOS = 4,      /* lks_check: positivity faults were counted      */
    LKS_ENAN = 5,         /* lks_check: a global sum is NaN                 */
    LKS_EUNSUPPORTED = 6  /* valid but not implemented combination          */
} lks_status;

enum { LKS_D2Q9 = 9, LKS_D2Q25 = 25 };
enum { LKS_F64 = 0, LKS_F32 = 1, LKS_BF16 = 2, LKS_F16 = 3 };
enum { LKS_PERIODIC = 0, LKS_OUTFLOW = 1 };
enum { LKS_LAYOUT_PLANES = 0, LKS_LAYOUT_ROWS = 1 };
enum { LKS_S_KL = 1u, LKS_S_NEQ = 2u, LKS_S_PI = 4u, LKS_S_Q = 8u, LKS_S_QE = 16u };

/* Kinetic model of a D2Q25 lattice (D2Q9 is always LKS_MODEL_BGK).
 *   LKS_MODEL_BGK  one distribution f (translational degrees of freedom only,
 *                  gamma = 2 in 2D), BGK collision, tau = mu/(rho T).
 *   LKS_MODEL_DDF  the double distribution of Sec. II.A.1-2: f carries mass,
 *                  momentum and translational energy, g the internal energy
 *                  of the non-translational degrees of freedom, g^eq =
 *                  (C_v - D/2) T f^eq (eq. energy_eq_1_rykov), C_v = 1/(gamma-1)
 *                  (R = 1), total energy E = sum g + sum |v|^2/2 f =
 *                  rho (C_v T + |u|^2/2).  Quasi-equilibrium collision with the
 *                  heat flux quasi-conserved (Pr <= 1, eq. new_collision_fi):
 *                  Omega = -(f - f*)/tau1 - (f* - f^eq)/tau2, likewise for g,
 *                  tau1 = mu/(rho T), tau2 = tau1/Pr; f* = f^eq + w_i (q_f . v_i)
 *                  (|v_i|^2/4 - 1) with the translational heat flux q_f =
 *                  1/2 sum |v - u|^2 (v - u) f, g* = g^eq + w_i (q_g . v_i) with
 *                  q_g = sum (v - u) g.  Both distributions take the same van
 *                  Leer fluxes.  State: 50 populations per cell (in the configured
 *                  layout), f deviations f_i - w_i rho0 (0..24), then g
 *                  deviations g_i - (C_v - 1) w_i rho0 (25..49).  Five sensor planes: 0 S_KL = |sum f
 *                  ln(f/f^eq)| + |sum g ln(g/g^eq)|, 1 S_NEQ = sum |f^neq| +
 *                  sum |g^neq|, 2 S_PI of f, 3 S_Q = |sum v g^neq + sum v |v|^2/2
 *                  f^neq|, 4 S_QE = sum |f* - f^eq| + sum |g* - g^eq| (eqs.
 *                  HKL-sensor, sensor-neq-kin, sensor-TauNS-kin,
 *                  sensor-qNSF-kin-ryk, Sensor-qe-kin); S_QE drives flag bit
 *                  LKS_S_QE with thresholds thr_qe.  A positivity fault is any
 *                  f, f^eq, g or g^eq not > 0.  The energy sum is E.  F32 or
 *                  F64 storage, fused steps.  Extension sensors (LKS_X_*,
 *                  planes after the five base planes) take the g terms
 *                  superposed and the QE collision as Omega: KN, HR, SIGMA_H,
 *                  SIGMA_HKL and ALPHA add the g form of each to the f form,
 *                  QF is |sum v g^neq + sum v |v|^2/2 f^neq - u . P|; SHEAR,
 *                  QH, COMP and STRAIN are those of f, COMP and STRAIN with
 *                  the model's second viscosity lambda = -(gamma - 1) mu and
 *                  bulk viscosity eta = 2 mu / D + lambda = (2 - gamma) mu
 *                  (Sec. II.A.2, eqs. viscHeating and visc_bluk_1 with
 *                  R/C_v = gamma - 1; Sec. III.A.2/4). */
enum { LKS_MODEL_BGK = 0, LKS_MODEL_DDF = 1 };

/* Extension sensors (bit k of ext_mask), the rest of Table I evaluated on the
 * f distribution in the same pass (with LKS_MODEL_DDF: f and g, see there),
 * on the pre-collision populations; BGK
 * collision Omega_i = -(f_i - f^eq_i)/tau, P = sum v v f^neq, q^neq =
 * sum v |v|^2/2 f^neq, u = sum v f / sum f; D2Q9 in lattice units with
 * mu = tau rho c_s^2 (c_s^2 = 1/3) and lambda = 0, D2Q25 with the configured
 * mu.  F32 or F64 storage and fused steps only.
 *   KN        sum |f^neq/f^eq|                    Sec. III.B.1, eq. sensor-Knudsen-kin_f
 *   HR        |H(f) - H(f^eq)|, H = sum f ln(f/w)  Sec. III.B.4, eq. Hneq-sensor (f term)
 *   SIGMA_H   -sum Omega ln(f/w)                  Sec. III.B.5, eq. Dissip-H-sensor (f term)
 *   SIGMA_HKL -sum Omega ln(f/f^eq)               Sec. III.B.5, eq. Dissip-HKL-sensor (f term)
 *   ALPHA     |2 - alpha_f|, the printed polynomial with f^neq = f - f^eq
 *                                                 Sec. III.B.6, eqs. sensor-alpha-kin,
 *                                                 alpha-polynomial-1/2
 *             Parity unpinned beyond leading order: the printed polynomial's
 *             first correction is -4 times that of the root of eq.
 *             H-mirr-equal, so these values agree with the entropic estimate
 *             in the limit f -> f^eq only (the sign and size of |2 - alpha|
 *             beyond that follow the printed coefficients).
 *   SHEAR     |(1/mu)[(tr P / D) I - P]|_F        Sec. III.A.3, eq. sensor-S-kin
 *   QH        |u . P|                             Sec. III.A.5, eq. sensor-qH-kin
 *   QF        |q^neq - u . P|  (D2Q25 only)       Sec. III.A.7, eq. sensor-qF-kin-ryk (g = 0)
 *   COMP      sqrt(D) |tr P| / |2 mu + D lambda|  Sec. III.A.2, eq. sensor-C-kin
 *             (D2Q9: lambda = 0; double distribution: see LKS_MODEL_DDF)
 *   STRAIN    |(1/2mu)[lambda/(D eta) tr(P) I - P]|_F, eta = 2 mu / D + lambda
 *                                                 Sec. III.A.4, eq. sensor-E-kin
 * COMP and STRAIN divide by 2 mu + D lambda and eta, which vanish for the
 * monatomic D2Q25 BGK gas (lambda = -mu): not available there; QF needs the
 * energy flux D2Q9 lacks.
 * Cells with a positivity fault get +inf for KN, HR, SIGMA_H, SIGMA_HKL and
 * ALPHA. */
#define LKS_MAX_EXT 10
enum {
    LKS_X_KN = 1u << 0, LKS_X_HR = 1u << 1, LKS_X_SIGMA_H = 1u << 2, LKS_X_SIGMA_HKL = 1u << 3,
    LKS_X_ALPHA = 1u << 4, LKS_X_SHEAR = 1u << 5, LKS_X_QH = 1u << 6, LKS_X_QF = 1u << 7,
    LKS_X_COMP = 1u << 8, LKS_X_STRAIN = 1u << 9
};
/* flag_mask bit of extension sensor k (k = 0 .. LKS_MAX_EXT-1) */
#define LKS_FLAG_X(k) (1u << (8 + (k)))

typedef struct {
    int32_t lattice;      /* LKS_D2Q9 or LKS_D2Q25                              */
    int32_t nx, ny;       /* grid size, >= 1 each (D2Q9 and periodic D2Q25
                             axes need no minimum; see lks_create)             */
    int32_t dtype;        /* population storage, LKS_F64..LKS_F16               */
    int32_t bc_x, bc_y;   /* D2Q25: LKS_PERIODIC or LKS_OUTFLOW (zero-gradient,
                             two ghost layers); D2Q9: must be LKS_PERIODIC     */
    double tau;           /* D2Q9 relaxation time in steps, > 0.5              */
    double mu, dt, dx;    /* D2Q25: dynamic viscosity, time step, cell size
                             (tau = mu/(rho T) per cell, R = 1); all > 0       */
    double rho0;          /* deviation reference density, > 0 (normally 1)     */
    uint32_t flag_mask;   /* sensors that drive the flags, LKS_S_* bits        */
    int32_t launch_rows;  /* rows per workgroup of the cell kernels; 0 picks
                             automatically (a launch-shape hint only)          */
    double thr[LKS_MAX_SENSORS][2]; /* (theta1 <= theta2) per sensor; compared
                             in the compute precision; +INF disables           */
    int32_t max_steps;    /* rows of the sums buffer, >= 1                     */
    int32_t launch_vec;   /* cells per thread along x of the cell kernels (1, 2
                             or 4); 0 picks 4 for F32 and 2 for the other
                             storage types, or fewer where the row length or
                             the buffer alignment do not allow it (a
                             launch-shape hint only)                           */
    uint32_t ext_mask;    /* extension sensors to compute and store, LKS_X_*
                             bits (0 = none)                                   */
    int32_t ext_reserved; /* must be 0                                          */
    double thr_ext[LKS_MAX_EXT][2]; /* (theta1 <= theta2) per extension sensor,
                             used when its LKS_FLAG_X bit is in flag_mask      */
    int32_t model;        /* LKS_MODEL_BGK (0) or, on D2Q25, LKS_MODEL_DDF     */
    int32_t layout;       /* population layout, LKS_LAYOUT_PLANES (0) or
                             LKS_LAYOUT_ROWS (see Conventions)                 */
    double gamma;         /* LKS_MODEL_DDF: adiabatic exponent, 1 < gamma < 2  */
    double prandtl;       /* LKS_MODEL_DDF: Prandtl number, 0 < Pr <= 1        */
    double thr_qe[2];     /* LKS_MODEL_DDF: (theta1 <= theta2) of S_QE         */
    int32_t launch_nt;    /* population stores of the fused step: 0 picks
                             (the non-temporal hint when the two state
                             buffers exceed the 256 MB last-level cache),
                             1 plain, 2 non-temporal (a launch hint only:
                             results are identical).  D2Q9 every storage
                             type; D2Q25 FP32 on grids of whole tiles      */
    int32_t launch_steps; /* fused D2Q9 steps per launch: 0 or 1 one, 2 two
                             (temporal blocking: the state crosses HBM once
                             per two steps; D2Q9 without extension sensors;
                             an odd last step of a reduction batch runs
                             alone in the one-step kernel; a batch holds at
                             most max_steps steps, so max_steps = 1 runs
                             every step in the one-step kernel).
                             A launch hint: state, sensors, flags and the
                             fault count are the same bits and the per-step
                             FP64 sums agree to FP64 rounding (each cell's
                             terms are widened to FP64 before any add), but
                             the state changes buffer once per launch, so
                             lks_current names the buffer that holds it      */
} lks_config;

typedef struct {
    void* pop[2];         /* Q*ny*nx values of dtype in the configured layout,
                             ping-pong state buffers (Q = 50 with
                             LKS_MODEL_DDF)                                    */
    void* sensors;        /* [lks_sensor_planes(cfg)][ny][nx] float (double for
                             F64): base planes, then the extension planes     */
    uint8_t* flags;       /* [ny][nx]                                          */
    double* sums;         /* [max_steps][LKS_NSUMS]                            */
    void* scratch;        /* >= lks_scratch_bytes(cfg) bytes, 256-B aligned    */
    size_t scratch_bytes;
} lks_buffers;

/* Device bytes of scratch the configuration needs (per-block FP64 partial
 * sums and counters; with LKS_MODEL_DDF also 6 values per cell that the
 * step's f kernel hands to its g kernel).  0 for an invalid configuration. */
size_t lks_scratch_bytes(const lks_config* cfg);

/* Number of base sensor planes of a lattice with the BGK model (3 for D2Q9,
 * 4 for D2Q25), 0 if invalid; LKS_MODEL_DDF has 5 (lks_sensor_planes). */
int32_t lks_num_sensors(int32_t lattice);

/* Sensor planes a configuration writes: the base planes plus one per
 * extension bit in ext_mask.  0 for an invalid configuration. */
int32_t lks_sensor_planes(const lks_config* cfg);

/* Validate cfg and buffers and create a context bound to hip_stream (a
 * hipStream_t; NULL = the null stream).  No kernel is launched. */
lks_status lks_create(const lks_config* cfg, const lks_buffers* buf, void* hip_stream,
                      lks_ctx** out);

/* Fill pop[0] with the equilibrium of the given FP64 device fields [ny][nx]
 * (the equilibrium initial condition of Sec. IV; with LKS_MODEL_DDF f^eq and
 * g^eq); T may be NULL on D2Q9 (isothermal) and is required on D2Q25.
 * Resets the step count to 0. */
lks_status lks_init_equilibrium(lks_ctx* ctx, const double* rho, const double* ux,
                                const double* uy, const double* T);

/* Declare that pop[pop_index] already holds a state (e.g. a copied-in
 * checkpoint) reached after steps_done steps. */
lks_status lks_restore(lks_ctx* ctx, int32_t pop_index, int64_t steps_done);

/* Advance nsteps (>= 0) steps.  fused = 1: one fused kernel per step (stream
 * or flux + collide + sensors + flags + sums).  fused = 0: the same result
 * from separate passes (D2Q9 only: stream into the other buffer, sensors and
 * flags, collide back), kept as the unfused baseline.  After the call
 * sensors and flags hold the last step's values. */
lks_status lks_step(lks_ctx* ctx, int32_t nsteps, int32_t fused);

/* ---- Stepping without allocation ----
 * For callers that cannot allocate memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  Does what
 * lks_restore(pop_index, steps_done) and then lks_step(nsteps, fused) do on a
 * context created from cfg and buf, without creating one: no host or device
 * memory is allocated.  cfg and buf are checked as by lks_create, except that
 * buf->scratch must be NULL and buf->scratch_bytes 0: the kernels' scratch
 * (fault counter, per-workgroup FP64 partial sums and, with LKS_MODEL_DDF,
 * the per-cell hand-over between the step's two kernels) is a device array
 * of LKS_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends (its address is looked up on the first call on a
 * device, with that device current).  A configuration whose scratch does not
 * fit (the hand-over plus one step's partial sums plus 256 bytes exceed the
 * array) returns LKS_EINVAL before anything is launched; the message (as for
 * lks_create, lks_last_error(NULL)) gives the bytes it needs.
 * The work is enqueued on hip_stream (a hipStream_t of the current device)
 * and the call returns without waiting.  *pop_index_out receives the index of
 * the buffer that holds the state after the call.  Populations, sensors,
 * flags and sums (step k of the call writes row (steps_done + k - 1) mod
 * max_steps) are those lks_step writes, bit for bit.  The positivity-fault
 * count is not reported (flag bit 7 marks the cells).
 * Every call on one GPU uses that GPU's one array, which keeps the last
 * call's contents (the fault counter is cleared at the start of each call):
 * calls that overlap on one GPU, from other streams or host threads, race on
 * it and must not be issued. */
#define LKS_NOALLOC_SCRATCH_BYTES (16u << 20)
lks_status lks_step_noalloc(const lks_config* cfg, const lks_buffers* buf, void* hip_stream,
                            int32_t pop_index, int64_t steps_done, int32_t nsteps, int32_t fused,
                            int32_t* pop_index_out);

/* One fused step from the state src into dst (both Q*ny*nx values in the
 * context's layout and dtype, distinct, neither need be pop[0]/pop[1]); sensors and
 * flags receive this step's values, the sums buffer and the step count are
 * left unchanged.  Used to recompute trajectory segments from checkpoints. */
lks_status lks_step_from(lks_ctx* ctx, const void* src, void* dst);

/* Index of the buffer holding the current state and the step count. */
lks_status lks_current(const lks_ctx* ctx, int32_t* pop_index, int64_t* steps_done);

/* Moments of the current state into FP64 device arrays [ny][nx]: rho, ux,
 * uy and, when T != NULL, the temperature (T_ref = 1/3 on D2Q9). */
lks_status lks_moments(lks_ctx* ctx, double* rho, double* ux, double* uy, double* T);

/* Synchronise the stream and copy to host memory: what = 0 current
 * populations (in the configured layout), 1 sensors, 2 flags, 3 sums.  bytes
 * must equal the buffer size. */
lks_status lks_read_host(lks_ctx* ctx, int32_t what, void* host_dst, size_t bytes);

/* Synchronise; report the number of positivity-fault cells counted since
 * init (LKS_ENONPOS if > 0) and LKS_ENAN if a stored sum of mass or momentum
 * is NaN. */
lks_status lks_check(lks_ctx* ctx, int64_t* n_nonpos);

/* ---- Adjoint of the D2Q9 step (gradient of the summed smooth KL sensor) ----
 * Loss L = sum_x S_KL(g_N(x)), g_N the pre-collision populations of the last
 * step N, initial populations at the equilibrium of (rho0, u0).  All arrays
 * are device populations (9 per cell, the context's layout and dtype, F32 or
 * F64) unless stated.
 *   seed:  lam_out = dL/dg_N, from pop_prev = f_{N-1} (the state before step N)
 *   step:  lam_out = dL/dg_n = J_C(g_n)^T S^T lam_in, lam_in = dL/dg_{n+1},
 *          pop_prev = f_{n-1}; J_C is the BGK collision Jacobian and S^T the
 *          adjoint of pull streaming (a pull by +c_i)
 *   init:  dL/du0 from lam0 = dL/dg_1 and the FP64 initial fields [ny][nx];
 *          writes FP64 gux, guy [ny][nx]. */
lks_status lks_adjoint_seed_kl(lks_ctx* ctx, const void* pop_prev, void* lam_out);
lks_status lks_adjoint_step(lks_ctx* ctx, const void* pop_prev, const void* lam_in,
                            void* lam_out);
lks_status lks_adjoint_init(lks_ctx* ctx, const double* rho0, const double* ux0,
                            const double* uy0, const void* lam0, double* gux, double* guy);

lks_status lks_destroy(lks_ctx* ctx);

const char* lks_status_str(lks_status s);

/* Message of the last failed call on ctx (or of the last failed lks_create
 * when ctx is NULL); valid until the next call on the same context. */
const char* lks_last_error(const lks_ctx* ctx);

/* ---- Macroscopic class-1 sensors (central differences) ----
 * The macroscopic counterparts of the class-1 sensors (Sec. III.A, eqs.
 * sensor-TauNS-mac, sensor-C-mac, sensor-S-mac, the rate-of-strain and
 * heat-flux forms), which the paper computes with central finite differences
 * to compare the kinetic sensors with (Sec. IV).  With A_ab = d_a u_b and
 * D = 2:
 *   LKS_M_TAU   |tau_NS|_F, tau_NS = -mu (A + A^T) - lambda (div u) I
 *   LKS_M_C     sqrt(D) |div u|
 *   LKS_M_S     |A + A^T - (2/D)(div u) I|_F
 *   LKS_M_E     |(A + A^T)/2|_F
 *   LKS_M_QH    |u . tau_NS|
 *   LKS_M_QF    |kappa grad T|
 *   LKS_M_QNSF  |-kappa grad T + u . tau_NS|
 * Derivatives (a[j+1] - a[j-1]) / (2 dx) with ghost cells by the context's
 * boundary conditions (periodic: wrap; outflow: repeat the edge cell); dx = 1
 * on D2Q9 (lattice units), the configured dx on D2Q25.  Inputs: FP64 device
 * fields [ny][nx] (e.g. those lks_moments writes); T is needed for QF and
 * QNSF, rho when transport->per_rho.  Transport: mu, lambda, kappa (finite),
 * each multiplied by the cell's density when per_rho != 0 (D2Q9 in lattice
 * units: mu = tau c_s^2).  out: FP64 device [popcount(which)][ny][nx], planes
 * in increasing bit order, distinct from the inputs.  Enqueued on the
 * context's stream; needs no state (no init). */
enum {
    LKS_M_TAU = 1u << 0, LKS_M_C = 1u << 1, LKS_M_S = 1u << 2, LKS_M_E = 1u << 3,
    LKS_M_QH = 1u << 4, LKS_M_QF = 1u << 5, LKS_M_QNSF = 1u << 6
};
typedef struct {
    double mu, lambda, kappa;
    int32_t per_rho;
    int32_t reserved;     /* must be 0 */
} lks_transport;
lks_status lks_macro_sensors(lks_ctx* ctx, const double* rho, const double* ux, const double* uy,
                             const double* T, const lks_transport* transport, uint32_t which,
                             double* out);

/* ---- Regridding hand-off (Sec. II.B.2, regridding steps 1-2) ----
 * The flag map is turned into refinement patches in three calls: a buffer
 * layer around the tagged cells (the paper uses two buffer cells, Sec. IV),
 * tag counts on blocking-factor tiles, and Berger-Rigoutsos clustering of the
 * tagged tiles into rectangles of a minimum grid efficiency (98 % in 2D in
 * the paper).  The first two run on the device on the context's stream; the
 * clustering runs on the host on the (small) tile counts. */
#define LKS_MAX_BUFFER 8

typedef struct {
    int32_t x0, y0, x1, y1;   /* cells [x0, x1) x [y0, y1) */
} lks_box;

/* Buffer layer: levels[c] = max over the (2b+1) x (2b+1) square around c of
 * (flags & 3), ghost cells by the context's boundary conditions (periodic:
 * wrap; outflow: the edge cell repeated).  flags, levels: device [ny][nx]
 * uint8 (they must not alias; flags may be the context's own flag buffer).
 * 0 <= b <= LKS_MAX_BUFFER, else LKS_EINVAL. */
lks_status lks_tag_buffer(lks_ctx* ctx, int32_t b, const uint8_t* flags, uint8_t* levels);

/* Tile counts: counts[t] = number of cells with (levels & 3) >= level in
 * tile t of ts x ts cells, tiles row-major [ceil(ny/ts)][ceil(nx/ts)] (the
 * high-edge tiles may be partial).  levels: device [ny][nx] uint8; counts:
 * device int32.  1 <= ts <= 64, 1 <= level <= 2, else LKS_EINVAL. */
lks_status lks_tag_tiles(lks_ctx* ctx, const uint8_t* levels, int32_t level, int32_t ts,
                         int32_t* counts);

/* Berger-Rigoutsos clustering (host): counts is a host array as written by
 * lks_tag_tiles for an nx x ny grid and tile size ts.  Boxes are tight
 * bounding boxes of tagged tiles, aligned to the tiles (clipped to the grid),
 * disjoint, covering every tagged tile, each with tagged cells >= eff x cells
 * unless no cut leaving min_tiles tiles on both sides exists.  Cuts: a hole
 * of a signature nearest the middle, else the strongest inflection of its
 * Laplacian, else halfway along the longer side (ties: x before y, lower
 * index).  Writes up to max_boxes boxes (depth-first order) and sets *nboxes
 * to the number found; LKS_EINVAL if that exceeds max_boxes or an argument
 * is invalid. */
lks_status lks_cluster(const int32_t* counts, int32_t nx, int32_t ny, int32_t ts, double eff,
                       int32_t min_tiles, lks_box* boxes, int32_t max_boxes, int32_t* nboxes);

/* Plain device-to-device copy of bytes (multiple of 16, 16-B aligned
 * pointers) on hip_stream: the bandwidth yardstick used to calibrate traffic
 * counters and the attainable HBM rate. */
lks_status lks_copy_probe(void* dst, const void* src, size_t bytes, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* LKS_H */
