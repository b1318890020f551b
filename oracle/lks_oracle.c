/*
 * lks_oracle.c -- plain FP64 CPU reference of the fused kinetic step with
 * local kinetic refinement sensors ("Local kinetic sensors for adaptive mesh
 * and algorithm refinement", arXiv 2603.13618).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or constant with the HIP
 * path: every constant below is derived here from its closed form.
 *
 * What it computes, in the paper's order and notation:
 *   - discrete velocities and weights from 1D Gauss-Hermite rules (Sec. II.A.3,
 *     "Discrete kinetic model"): D2Q9 = GH3 x GH3 scaled by sqrt(T_ref),
 *     T_ref = 1/3; D2Q25 = GH5 x GH5, T_ref = 1;
 *   - moments as quadratures (Sec. II.A.3, eq. quadratur1/2, eq. for E with the
 *     translational part only, i.e. no g population);
 *   - Grad-Hermite equilibria to order N (Sec. II.A.3, the expansion of
 *     f^eq_i in Hermite tensors): N = 2 on D2Q9 (isothermal), N = 4 on D2Q25;
 *   - D2Q9: lattice-BGK pull streaming g_i(x) = f_i(x - c_i) on a periodic
 *     grid, then single-relaxation BGK f' = g - (g - f^eq)/tau (the QE
 *     collision of Sec. II.A.1 with tau1 = tau2);
 *   - D2Q25: the explicit-Euler finite-volume update eq. finalDiscretePDE with
 *     dimension-by-dimension upwind fluxes, a van Leer limited linear
 *     reconstruction (Sec. II.A.3, last paragraph) and BGK relaxation with
 *     tau = mu/(rho T) (Sec. II.A.2, NSF limit, mu = tau p with p = rho R T);
 *   - sensors on the pre-collision populations of each step:
 *       S_KL  = sum_i f_i ln(f_i/f^eq_i)            (Sec. III.B.5, eq. HKL-sensor, f term)
 *               evaluated term by term as f^eq_i [(1+x_i) ln(1+x_i) - x_i] with
 *               x_i = f^neq_i / f^eq_i, i.e. f_i ln(f_i/f^eq_i) - f_i + f^eq_i,
 *               which sums to the same number because sum_i f_i = sum_i f^eq_i
 *               = rho, and has no round-off floor at equilibrium;
 *       S_NEQ = sum_i |f_i - f^eq_i|                  (Sec. III.B.2, eq. sensor-neq-kin, f term)
 *       S_PI  = || sum_i v_i v_i f^neq_i ||_F          (Sec. III.A.1, eq. sensor-TauNS-kin)
 *       S_Q   = || sum_i v_i (|v_i|^2/2) f^neq_i ||_2  (Sec. III.A.6, eq. sensor-qNSF-kin-ryk, g = 0)
 *   - extended sensors on demand (orc_ext_sensors): the rest of Table I on
 *     the f distribution -- Knudsen, relative H, H dissipation, KL
 *     dissipation, entropic estimate, rate of shear, viscous heating, Fourier
 *     flux (D2Q25), rate of compression and rate of strain (D2Q9).  The
 *     entropic estimate is parity unpinned beyond leading order: the printed
 *     polynomial (eqs. alpha-polynomial-1/2) has a first correction -4 times
 *     that of the root of its defining condition (eq. H-mirr-equal), and is
 *     evaluated as printed;
 *   - refinement flags (Sec. II.B.2, regridding step 1): per enabled sensor
 *     level = [s > theta1] + [s > theta2]; flag = max over sensors; a cell
 *     whose f_i or f^eq_i is not strictly positive (Sec. III.C, positivity
 *     caveat) gets S_KL = +inf and flag = 2 | 0x80;
 *   - FP64 global sums of the pre-collision state: mass, momentum, energy
 *     (D2Q25) and the sensor totals.
 *
 * Plain loops over cells; OpenMP splits rows only (each cell is independent,
 * per-row partial sums are added in fixed row order, so results do not depend
 * on the thread count).
 *
 * Layout: structure of arrays, f[i][y][x], x fastest, population index
 * i = q1*a + b with a the x-node and b the y-node index, nodes ascending.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_NSUMS 8
#define ORC_MAXQ1 5
#define ORC_MAXQ (ORC_MAXQ1 * ORC_MAXQ1)

/* ------------------------------------------------------------------------ */
/* 1D Gauss-Hermite rules and Hermite polynomials                            */
/* ------------------------------------------------------------------------ */

typedef struct {
    int q1;                 /* nodes per axis                               */
    int order;              /* Grad-Hermite truncation order N              */
    double tref;            /* lattice reference temperature T_ref (R = 1)  */
    double xi[ORC_MAXQ1];   /* nodes of the rule with weight exp(-x^2/2)    */
    double w[ORC_MAXQ1];    /* normalised weights, sum = 1                  */
    double v[ORC_MAXQ1];    /* physical velocity component sqrt(T_ref)*xi   */
    double he[ORC_MAXQ1][ORC_MAXQ1]; /* He_n(xi_a) / n!, filled by rule_finish */
} orc_rule;

static double hermite_he(int n, double x);
static double factorial(int n);

/* table of He_n(xi_a) / n! for the Grad-Hermite sums */
static void rule_finish(orc_rule* r)
{
    for (int a = 0; a < r->q1; ++a)
        for (int n = 0; n <= r->order; ++n)
            r->he[a][n] = hermite_he(n, r->xi[a]) / factorial(n);
}

/* GH3: roots of He_3 = x^3 - 3x are 0, +-sqrt(3); weights 2/3, 1/6.
 * D2Q9 uses the integer velocities -1, 0, 1 = sqrt(1/3) * (-sqrt3, 0, sqrt3). */
static void rule_d2q9(orc_rule* r)
{
    r->q1 = 3;
    r->order = 2;
    r->tref = 1.0 / 3.0;
    const double c[3] = {-1.0, 0.0, 1.0};
    for (int a = 0; a < 3; ++a) {
        r->v[a] = c[a];
        r->xi[a] = c[a] * sqrt(3.0);
    }
    r->w[0] = 1.0 / 6.0;
    r->w[1] = 2.0 / 3.0;
    r->w[2] = 1.0 / 6.0;
    rule_finish(r);
}

/* GH5: roots of He_5 = x^5 - 10x^3 + 15x are 0 and x^2 = 5 -+ sqrt(10);
 * weights 8/15 and (7 -+ 2 sqrt(10))/60 for the outer/inner pairs. */
static void rule_d2q25(orc_rule* r)
{
    r->q1 = 5;
    r->order = 4;
    r->tref = 1.0;
    const double s10 = sqrt(10.0);
    const double xo = sqrt(5.0 + s10), xn = sqrt(5.0 - s10);
    const double wo = (7.0 - 2.0 * s10) / 60.0, wn = (7.0 + 2.0 * s10) / 60.0;
    r->xi[0] = -xo; r->w[0] = wo;
    r->xi[1] = -xn; r->w[1] = wn;
    r->xi[2] = 0.0; r->w[2] = 8.0 / 15.0;
    r->xi[3] = xn;  r->w[3] = wn;
    r->xi[4] = xo;  r->w[4] = wo;
    for (int a = 0; a < 5; ++a) r->v[a] = r->xi[a] * sqrt(r->tref);
    rule_finish(r);
}

/* probabilists' Hermite polynomial He_n by the three-term recurrence */
static double hermite_he(int n, double x)
{
    double hm = 1.0, h = x;
    if (n == 0) return 1.0;
    for (int k = 1; k < n; ++k) {
        double hp = x * h - (double)k * hm;
        hm = h;
        h = hp;
    }
    return h;
}

static double factorial(int n)
{
    double r = 1.0;
    for (int k = 2; k <= n; ++k) r *= (double)k;
    return r;
}

/* Hermite coefficient of a 1D Gaussian of mean u and variance theta in units
 * of T_ref: h_n = E[He_n(X)], X ~ N(u, theta)
 *      = sum_k n! / (k! (n-2k)! 2^k) u^(n-2k) (theta - 1)^k. */
static double gauss_hermite_coeff(int n, double u, double theta)
{
    double s = 0.0;
    for (int k = 0; 2 * k <= n; ++k)
        s += factorial(n) / (factorial(k) * factorial(n - 2 * k) * pow(2.0, k))
           * pow(u, n - 2 * k) * pow(theta - 1.0, k);
    return s;
}

/* Grad-Hermite equilibrium to order N (Sec. II.A.3):
 * f^eq_i = w_i sum_{n<=N} a_n : H_n(xi_i) / n!  with the Maxwellian's
 * coefficients; in 2D the n-th tensor contraction splits into the products
 * a_(nx,ny) He_nx(xi_a) He_ny(xi_b) / (nx! ny!), nx + ny = n, and the
 * Maxwellian's a_(nx,ny) = rho h_nx(ux~) h_ny(uy~) with u~ = u/sqrt(T_ref),
 * theta = T/T_ref. */
static void grad_hermite_feq(const orc_rule* r, double rho, double ux, double uy, double T,
                             double* feq)
{
    const double s = sqrt(r->tref);
    const double utx = ux / s, uty = uy / s, th = T / r->tref;
    double hx[ORC_MAXQ1], hy[ORC_MAXQ1];
    for (int n = 0; n <= r->order; ++n) {
        hx[n] = gauss_hermite_coeff(n, utx, th);
        hy[n] = gauss_hermite_coeff(n, uty, th);
    }
    for (int a = 0; a < r->q1; ++a)
        for (int b = 0; b < r->q1; ++b) {
            double sum = 0.0;
            for (int nx = 0; nx <= r->order; ++nx)
                for (int ny = 0; nx + ny <= r->order; ++ny)
                    sum += hx[nx] * hy[ny] * r->he[a][nx] * r->he[b][ny];
            feq[r->q1 * a + b] = r->w[a] * r->w[b] * rho * sum;
        }
}

/* ------------------------------------------------------------------------ */
/* Cell-local pieces shared by both steppers                                  */
/* ------------------------------------------------------------------------ */

typedef struct {
    double rho, jx, jy, E, ux, uy, T;
} orc_mom;

/* quadrature moments (Sec. II.A.3): rho = sum f, rho u = sum v f,
 * E = sum |v|^2/2 f (translational energy only: no g population);
 * T = (2E/rho - |u|^2)/D with D = 2 (monatomic 2D gas, R = 1). */
static orc_mom moments(const orc_rule* r, const double* f)
{
    orc_mom m = {0, 0, 0, 0, 0, 0, 0};
    for (int a = 0; a < r->q1; ++a)
        for (int b = 0; b < r->q1; ++b) {
            const double fi = f[r->q1 * a + b];
            m.rho += fi;
            m.jx += r->v[a] * fi;
            m.jy += r->v[b] * fi;
            m.E += 0.5 * (r->v[a] * r->v[a] + r->v[b] * r->v[b]) * fi;
        }
    m.ux = m.jx / m.rho;
    m.uy = m.jy / m.rho;
    m.T = (2.0 * m.E / m.rho - (m.ux * m.ux + m.uy * m.uy)) / 2.0;
    return m;
}

/* sensors of one cell: s[0] = S_KL, s[1] = S_NEQ, s[2] = S_PI, s[3] = S_Q.
 * Returns 1 when a population or equilibrium is not strictly positive. */
static int cell_sensors(const orc_rule* r, const double* f, const double* feq, int with_q,
                        double* s)
{
    int fault = 0;
    double kl = 0.0, neq = 0.0, pxx = 0.0, pxy = 0.0, pyy = 0.0, qx = 0.0, qy = 0.0;
    for (int a = 0; a < r->q1; ++a)
        for (int b = 0; b < r->q1; ++b) {
            const int i = r->q1 * a + b;
            const double fn = f[i] - feq[i];
            const double vx = r->v[a], vy = r->v[b];
            if (!(f[i] > 0.0) || !(feq[i] > 0.0)) {
                fault = 1;
            } else {
                const double x = fn / feq[i];
                kl += feq[i] * ((1.0 + x) * log1p(x) - x);
            }
            neq += fabs(fn);
            pxx += vx * vx * fn;
            pxy += vx * vy * fn;
            pyy += vy * vy * fn;
            const double e = 0.5 * (vx * vx + vy * vy);
            qx += vx * e * fn;
            qy += vy * e * fn;
        }
    s[0] = fault ? INFINITY : kl;
    s[1] = neq;
    s[2] = sqrt(pxx * pxx + 2.0 * pxy * pxy + pyy * pyy);
    s[3] = with_q ? sqrt(qx * qx + qy * qy) : 0.0;
    return fault;
}

/* flag of one cell from its sensors and the thresholds thr[k][0..1] */
static uint8_t cell_flag(const double* s, const double* thr, unsigned mask, int fault)
{
    int level = 0;
    for (int k = 0; k < 4; ++k) {
        if (!(mask & (1u << k))) continue;
        const int l = (s[k] > thr[2 * k]) + (s[k] > thr[2 * k + 1]);
        if (l > level) level = l;
    }
    if (fault) return (uint8_t)(2 | 0x80);
    return (uint8_t)level;
}

/* ------------------------------------------------------------------------ */
/* Public helpers                                                            */
/* ------------------------------------------------------------------------ */

/* lattice: 9 or 25.  Writes Q velocities (vx, vy) and weights. */
int orc_lattice(int lattice, double* vx, double* vy, double* w)
{
    orc_rule r;
    if (lattice == 9) rule_d2q9(&r);
    else if (lattice == 25) rule_d2q25(&r);
    else return -1;
    for (int a = 0; a < r.q1; ++a)
        for (int b = 0; b < r.q1; ++b) {
            const int i = r.q1 * a + b;
            vx[i] = r.v[a];
            vy[i] = r.v[b];
            w[i] = r.w[a] * r.w[b];
        }
    return r.q1 * r.q1;
}

/* equilibrium populations for n cells (T ignored on D2Q9: isothermal,
 * T = T_ref).  feq is [Q][n]. */
int orc_equilibrium(int lattice, long n, const double* rho, const double* ux, const double* uy,
                    const double* T, double* feq)
{
    orc_rule r;
    if (lattice == 9) rule_d2q9(&r);
    else if (lattice == 25) rule_d2q25(&r);
    else return -1;
    const int Q = r.q1 * r.q1;
#pragma omp parallel for schedule(static)
    for (long c = 0; c < n; ++c) {
        double fe[ORC_MAXQ];
        const double Tc = (lattice == 9 || T == NULL) ? r.tref : T[c];
        grad_hermite_feq(&r, rho[c], ux[c], uy[c], Tc, fe);
        for (int i = 0; i < Q; ++i) feq[(long)i * n + c] = fe[i];
    }
    return 0;
}

/* moments of n cells: out[0..3][n] = rho, ux, uy, T */
int orc_moments(int lattice, long n, const double* f, double* out)
{
    orc_rule r;
    if (lattice == 9) rule_d2q9(&r);
    else if (lattice == 25) rule_d2q25(&r);
    else return -1;
    const int Q = r.q1 * r.q1;
#pragma omp parallel for schedule(static)
    for (long c = 0; c < n; ++c) {
        double fc[ORC_MAXQ];
        for (int i = 0; i < Q; ++i) fc[i] = f[(long)i * n + c];
        orc_mom m = moments(&r, fc);
        out[c] = m.rho;
        out[n + c] = m.ux;
        out[2 * n + c] = m.uy;
        out[3 * n + c] = (lattice == 9) ? r.tref : m.T;
    }
    return 0;
}

/* sensors of n cells given their populations f[Q][n]: out[4][n]; the
 * equilibrium is built from the cells' own moments.  Returns the number of
 * cells with a positivity fault. */
long orc_sensors(int lattice, long n, const double* f, double* out)
{
    orc_rule r;
    if (lattice == 9) rule_d2q9(&r);
    else if (lattice == 25) rule_d2q25(&r);
    else return -1;
    const int Q = r.q1 * r.q1;
    long faults = 0;
#pragma omp parallel for schedule(static) reduction(+ : faults)
    for (long c = 0; c < n; ++c) {
        double fc[ORC_MAXQ], fe[ORC_MAXQ], s[4];
        for (int i = 0; i < Q; ++i) fc[i] = f[(long)i * n + c];
        orc_mom m = moments(&r, fc);
        grad_hermite_feq(&r, m.rho, m.ux, m.uy, lattice == 9 ? r.tref : m.T, fe);
        faults += cell_sensors(&r, fc, fe, lattice == 25, s);
        for (int k = 0; k < 4; ++k) out[(long)k * n + c] = s[k];
    }
    return faults;
}

/* ------------------------------------------------------------------------ */
/* Extended sensors (the rest of Table I on the f distribution)             */
/* ------------------------------------------------------------------------ */

/* Order of the extended sensor planes. */
enum {
    ORC_X_KN = 0,      /* sum |f^neq/f^eq|                  (Sec. III.B.1, eq. sensor-Knudsen-kin_f)   */
    ORC_X_HR,          /* |H(f) - H(f^eq)|, H = sum f ln(f/w)  (Sec. III.B.4, eq. Hneq-sensor, f term)  */
    ORC_X_SIGMA_H,     /* -sum Omega ln(f/w)                 (Sec. III.B.5, eq. Dissip-H-sensor)        */
    ORC_X_SIGMA_HKL,   /* -sum Omega ln(f/f^eq)              (Sec. III.B.5, eq. Dissip-HKL-sensor)      */
    ORC_X_ALPHA,       /* |2 - alpha_f|, polynomial estimate (Sec. III.B.6, eqs. sensor-alpha-kin,
                          alpha-polynomial-1/2)                                                         */
    ORC_X_SHEAR,       /* |(1/mu)[(1/D) tr(P) I - P]|_F      (Sec. III.A.3, eq. sensor-S-kin)           */
    ORC_X_QH,          /* |u . P|                            (Sec. III.A.5, eq. sensor-qH-kin)          */
    ORC_X_QF,          /* |q^neq - u . P| (D2Q25)            (Sec. III.A.7, eq. sensor-qF-kin-ryk, g=0) */
    ORC_X_COMP,        /* sqrt(D)|tr P|/|2 mu + D lambda| (D2Q9) (Sec. III.A.2, eq. sensor-C-kin)        */
    ORC_X_STRAIN,      /* |(1/2mu)[lambda/(D eta) tr(P) I - P]|_F (D2Q9) (Sec. III.A.4, eq. sensor-E-kin) */
    ORC_NEXT
};

/* Extended sensors of one cell from its populations f and equilibrium feq.
 * P = sum v v f^neq, q^neq = sum v |v|^2/2 f^neq, u = sum v f / sum f.
 * The collision is single-relaxation BGK, Omega_i = -(f_i - f^eq_i)/tau, with
 * tau the lattice relaxation time on D2Q9 and mu/(rho T) on D2Q25.
 * Viscosities: on D2Q25 mu is the model's dynamic viscosity; the monatomic
 * gas (C_v = D R/2) has lambda = -mu and eta = 0, so the rate-of-compression
 * and rate-of-strain sensors have a zero denominator there and are not
 * defined (left 0).  On the isothermal D2Q9 lattice the pre-collision
 * non-equilibrium stress is -tau rho c_s^2 (grad u + grad u^T) with no
 * separate trace term, i.e. mu = tau rho c_s^2 and lambda = 0 (eta = mu).
 * Cells with f_i <= 0 or f^eq_i <= 0 get +inf for the five sensors that
 * take logarithms or ratios of populations.
 * The entropic estimate follows the printed polynomial with f^neq = f - f^eq
 * as the paper defines it.  That polynomial is not the series solution of
 * its defining condition (eq. H-mirr-equal): the exact root is
 * alpha = 2 - (1/3) sum f^neq^3/f^2 / sum f^neq^2/f + O(y^2), the polynomial's
 * first correction is -4 times that, and the higher terms differ in structure.
 * Parity unpinned beyond leading order: only the printed text fixes the
 * r2^2, r3 and higher coefficients, and the paper is at odds with itself
 * there.  |2 - alpha_f| = 0 when a_1 = 0. */
static void cell_ext_sensors(const orc_rule* r, const double* f, const double* feq, int lattice,
                             double par, double* s)
{
    const int D = 2;
    double rho = 0.0, jx = 0.0, jy = 0.0;
    double kn = 0.0, hf = 0.0, heq = 0.0, sig_h = 0.0, sig_hkl = 0.0;
    double an[5] = {0, 0, 0, 0, 0};
    double pxx = 0.0, pxy = 0.0, pyy = 0.0, qx = 0.0, qy = 0.0;
    int fault = 0;
    for (int a = 0; a < r->q1; ++a)
        for (int b = 0; b < r->q1; ++b) {
            const int i = r->q1 * a + b;
            const double vx = r->v[a], vy = r->v[b];
            rho += f[i];
            jx += vx * f[i];
            jy += vy * f[i];
            const double fn = f[i] - feq[i];
            pxx += vx * vx * fn;
            pxy += vx * vy * fn;
            pyy += vy * vy * fn;
            const double e = 0.5 * (vx * vx + vy * vy);
            qx += vx * e * fn;
            qy += vy * e * fn;
        }
    const double ux = jx / rho, uy = jy / rho;
    /* relaxation time and viscosity */
    double tau, mu;
    if (lattice == 9) {
        tau = par;
        mu = tau * rho * r->tref;
    } else {
        const orc_mom m = moments(r, f);
        mu = par;
        tau = mu / (m.rho * m.T);
    }
    for (int a = 0; a < r->q1; ++a)
        for (int b = 0; b < r->q1; ++b) {
            const int i = r->q1 * a + b;
            const double w = r->w[a] * r->w[b];
            if (!(f[i] > 0.0) || !(feq[i] > 0.0)) {
                fault = 1;
                continue;
            }
            const double fn = f[i] - feq[i];
            const double omega = -fn / tau;
            kn += fabs(fn / feq[i]);
            hf += f[i] * log(f[i] / w);
            heq += feq[i] * log(feq[i] / w);
            sig_h -= omega * log(f[i] / w);
            sig_hkl -= omega * log(f[i] / feq[i]);
            for (int n = 1; n <= 4; ++n) an[n] += pow(fn, n + 1) / pow(f[i], n);
        }
    for (int n = 1; n <= 4; ++n) an[n] *= ((n % 2) ? 1.0 : -1.0) / (n * (n + 1.0));
    double alpha_dev = 0.0;           /* 2 - alpha_f */
    if (an[1] != 0.0) {
        const double r2 = an[2] / an[1], r3 = an[3] / an[1], r4 = an[4] / an[1];
        const double alpha = 2.0 - 4.0 * r2 + 16.0 * r2 * r2 - 8.0 * r3 + 80.0 * r2 * r3
                             - 80.0 * r2 * r2 * r2 - 16.0 * r4;
        alpha_dev = 2.0 - alpha;
    }
    const double tr = pxx + pyy;
    /* rate of shear: (1/mu) [(tr/D) I - P] */
    const double sxx = (tr / D - pxx) / mu, syy = (tr / D - pyy) / mu, sxy = -pxy / mu;
    /* viscous heating u . P and the Fourier part q^neq - u . P */
    const double hx = ux * pxx + uy * pxy, hy = ux * pxy + uy * pyy;
    s[ORC_X_KN] = fault ? INFINITY : kn;
    s[ORC_X_HR] = fault ? INFINITY : fabs(hf - heq);
    s[ORC_X_SIGMA_H] = fault ? INFINITY : sig_h;
    s[ORC_X_SIGMA_HKL] = fault ? INFINITY : sig_hkl;
    s[ORC_X_ALPHA] = fault ? INFINITY : fabs(alpha_dev);
    s[ORC_X_SHEAR] = sqrt(sxx * sxx + 2.0 * sxy * sxy + syy * syy);
    s[ORC_X_QH] = sqrt(hx * hx + hy * hy);
    if (lattice == 25) {
        s[ORC_X_QF] = sqrt((qx - hx) * (qx - hx) + (qy - hy) * (qy - hy));
        s[ORC_X_COMP] = 0.0;
        s[ORC_X_STRAIN] = 0.0;
    } else {
        const double lambda = 0.0, eta = 2.0 * mu / D + lambda;
        s[ORC_X_QF] = 0.0;
        s[ORC_X_COMP] = sqrt((double)D) * fabs(tr) / fabs(2.0 * mu + D * lambda);
        const double c = lambda / (D * eta);
        const double exx = (c * tr - pxx) / (2.0 * mu), eyy = (c * tr - pyy) / (2.0 * mu),
                     exy = -pxy / (2.0 * mu);
        s[ORC_X_STRAIN] = sqrt(exx * exx + 2.0 * exy * exy + eyy * eyy);
    }
}

int orc_num_ext(void) { return ORC_NEXT; }

/* Extended sensors of n cells given their (pre-collision) populations
 * f[Q][n]: out[ORC_NEXT][n].  par = tau on D2Q9, mu on D2Q25.  The
 * equilibrium is built from each cell's own moments. */
int orc_ext_sensors(int lattice, long n, const double* f, double par, double* out)
{
    orc_rule r;
    if (lattice == 9) rule_d2q9(&r);
    else if (lattice == 25) rule_d2q25(&r);
    else return -1;
    const int Q = r.q1 * r.q1;
#pragma omp parallel for schedule(static)
    for (long c = 0; c < n; ++c) {
        double fc[ORC_MAXQ], fe[ORC_MAXQ], s[ORC_NEXT];
        for (int i = 0; i < Q; ++i) fc[i] = f[(long)i * n + c];
        orc_mom m = moments(&r, fc);
        grad_hermite_feq(&r, m.rho, m.ux, m.uy, lattice == 9 ? r.tref : m.T, fe);
        cell_ext_sensors(&r, fc, fe, lattice, par, s);
        for (int k = 0; k < ORC_NEXT; ++k) out[(long)k * n + c] = s[k];
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* D2Q9 lattice-BGK step                                                      */
/* ------------------------------------------------------------------------ */

static inline long wrap(long j, long n)
{
    j %= n;
    return j < 0 ? j + n : j;
}

/* One step: pull-stream f -> g (periodic), then per cell moments,
 * equilibrium, sensors, flag and BGK collision into fout.
 * Optional outputs (NULL to skip): g [9][n], mom [4][n] (rho, ux, uy, T of
 * the pre-collision state), sens [4][n], flags [n].  sums[8] always:
 * total mass, x/y momentum, 0 (no energy on D2Q9), sensor totals.
 * Returns the number of cells with a positivity fault. */
long orc_d2q9_step(int nx, int ny, double tau, const double* f, double* fout, double* g_out,
                   double* mom, double* sens, uint8_t* flags, const double* thr, unsigned mask,
                   double* sums)
{
    orc_rule r;
    rule_d2q9(&r);
    const long n = (long)nx * ny;
    double* g = g_out ? g_out : (double*)malloc(sizeof(double) * 9 * (size_t)n);
    double* rowsum = (double*)calloc((size_t)ny * ORC_NSUMS, sizeof(double));
    long faults = 0;

    /* streaming: g_i(x) = f_i(x - c_i) */
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            const int i = 3 * a + b;
            const int cx = a - 1, cy = b - 1;
#pragma omp parallel for schedule(static)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x)
                    g[(long)i * n + (long)y * nx + x] =
                        f[(long)i * n + wrap(y - cy, ny) * nx + wrap(x - cx, nx)];
        }

#pragma omp parallel for schedule(static) reduction(+ : faults)
    for (int y = 0; y < ny; ++y) {
        double* rs = rowsum + (size_t)y * ORC_NSUMS;
        for (int x = 0; x < nx; ++x) {
            const long c = (long)y * nx + x;
            double gc[9], fe[9], s[4];
            for (int i = 0; i < 9; ++i) gc[i] = g[(long)i * n + c];
            const orc_mom m = moments(&r, gc);
            grad_hermite_feq(&r, m.rho, m.ux, m.uy, r.tref, fe);
            const int fault = cell_sensors(&r, gc, fe, 0, s);
            faults += fault;
            for (int i = 0; i < 9; ++i) fout[(long)i * n + c] = gc[i] - (gc[i] - fe[i]) / tau;
            if (mom) {
                mom[c] = m.rho;
                mom[n + c] = m.ux;
                mom[2 * n + c] = m.uy;
                mom[3 * n + c] = r.tref;
            }
            if (sens)
                for (int k = 0; k < 4; ++k) sens[(long)k * n + c] = s[k];
            if (flags) flags[c] = cell_flag(s, thr, mask, fault);
            rs[0] += m.rho;
            rs[1] += m.jx;
            rs[2] += m.jy;
            for (int k = 0; k < 4; ++k) rs[4 + k] += s[k];
        }
    }
    for (int k = 0; k < ORC_NSUMS; ++k) sums[k] = 0.0;
    for (int y = 0; y < ny; ++y)
        for (int k = 0; k < ORC_NSUMS; ++k) sums[k] += rowsum[(size_t)y * ORC_NSUMS + k];
    free(rowsum);
    if (!g_out) free(g);
    return faults;
}

/* ------------------------------------------------------------------------ */
/* D2Q25 finite-volume step                                                   */
/* ------------------------------------------------------------------------ */

/* ghost-cell index: bc 0 = periodic, 1 = zero-gradient outflow (the ghost
 * layers repeat the boundary cell) */
static inline long ghost(long j, long n, int bc)
{
    if (bc == 0) return wrap(j, n);
    return j < 0 ? 0 : (j >= n ? n - 1 : j);
}

/* van Leer limited slope of the differences a (backward) and b (forward):
 * 2ab/(a+b) when a and b have the same strict sign, else 0 */
static inline double van_leer(double a, double b)
{
    return (a * b > 0.0) ? 2.0 * a * b / (a + b) : 0.0;
}

/* upwind flux v * f_face through the face between cells j and j+1, from the
 * four cell values q[j-1], q[j], q[j+1], q[j+2] */
static inline double face_flux(double v, double qm1, double q0, double q1, double q2)
{
    if (v > 0.0) return v * (q0 + 0.5 * van_leer(q0 - qm1, q1 - q0));
    if (v < 0.0) return v * (q1 - 0.5 * van_leer(q1 - q0, q2 - q1));
    return 0.0;
}

/* One explicit-Euler FV step (eq. finalDiscretePDE):
 *   f^{n+1} = f^n - dt/dx * sum_faces F + dt/tau (f^eq - f^n),
 * tau = mu / (rho T).  Sensors, flags and sums are of f^n, the state the
 * collision reads.  bc_x, bc_y: 0 periodic, 1 outflow.  Optional outputs as
 * for the D2Q9 step; mom holds rho, ux, uy, T. */
long orc_d2q25_step(int nx, int ny, double mu, double dt, double dx, int bc_x, int bc_y,
                    const double* f, double* fout, double* mom, double* sens, uint8_t* flags,
                    const double* thr, unsigned mask, double* sums)
{
    orc_rule r;
    rule_d2q25(&r);
    const long n = (long)nx * ny;
    double* rowsum = (double*)calloc((size_t)ny * ORC_NSUMS, sizeof(double));
    long faults = 0;

#pragma omp parallel for schedule(static) reduction(+ : faults)
    for (int y = 0; y < ny; ++y) {
        double* rs = rowsum + (size_t)y * ORC_NSUMS;
        for (int x = 0; x < nx; ++x) {
            const long c = (long)y * nx + x;
            double fc[25], fe[25], s[4];
            for (int i = 0; i < 25; ++i) fc[i] = f[(long)i * n + c];
            const orc_mom m = moments(&r, fc);
            grad_hermite_feq(&r, m.rho, m.ux, m.uy, m.T, fe);
            const int fault = cell_sensors(&r, fc, fe, 1, s);
            faults += fault;
            const double tau = mu / (m.rho * m.T);
            for (int a = 0; a < 5; ++a)
                for (int b = 0; b < 5; ++b) {
                    const int i = 5 * a + b;
                    const double* fi = f + (long)i * n;
                    const double vx = r.v[a], vy = r.v[b];
                    double div = 0.0;
                    if (vx != 0.0) {
                        double q[5];
                        for (int k = -2; k <= 2; ++k)
                            q[k + 2] = fi[(long)y * nx + ghost(x + k, nx, bc_x)];
                        const double fr = face_flux(vx, q[1], q[2], q[3], q[4]);
                        const double fl = face_flux(vx, q[0], q[1], q[2], q[3]);
                        div += (fr - fl) / dx;
                    }
                    if (vy != 0.0) {
                        double q[5];
                        for (int k = -2; k <= 2; ++k)
                            q[k + 2] = fi[ghost(y + k, ny, bc_y) * nx + x];
                        const double fr = face_flux(vy, q[1], q[2], q[3], q[4]);
                        const double fl = face_flux(vy, q[0], q[1], q[2], q[3]);
                        div += (fr - fl) / dx;
                    }
                    fout[(long)i * n + c] = fc[i] - dt * div + (dt / tau) * (fe[i] - fc[i]);
                }
            if (mom) {
                mom[c] = m.rho;
                mom[n + c] = m.ux;
                mom[2 * n + c] = m.uy;
                mom[3 * n + c] = m.T;
            }
            if (sens)
                for (int k = 0; k < 4; ++k) sens[(long)k * n + c] = s[k];
            if (flags) flags[c] = cell_flag(s, thr, mask, fault);
            rs[0] += m.rho;
            rs[1] += m.jx;
            rs[2] += m.jy;
            rs[3] += m.E;
            for (int k = 0; k < 4; ++k) rs[4 + k] += s[k];
        }
    }
    for (int k = 0; k < ORC_NSUMS; ++k) sums[k] = 0.0;
    for (int y = 0; y < ny; ++y)
        for (int k = 0; k < ORC_NSUMS; ++k) sums[k] += rowsum[(size_t)y * ORC_NSUMS + k];
    free(rowsum);
    return faults;
}

/* ------------------------------------------------------------------------ */
/* D2Q25 double distribution (f, g) with the quasi-equilibrium collision     */
/* ------------------------------------------------------------------------ */
/*
 * The paper's kinetic model (Sec. II.A.1-2): f carries mass, momentum and the
 * translational energy, g the non-translational internal energy (the
 * internal non-translational split, eq. energy_eq_1_rykov):
 *   rho = sum f, rho u = sum v f, E = sum (g + |v|^2/2 f) = rho C_v T + rho |u|^2/2,
 *   g^eq = (C_v - R D/2) T f^eq, C_v = R/(gamma - 1), R = 1, D = 2.
 * Collision (eq. new_collision_fi): Omega = -(f - f*)/tau1 - (f* - f^eq)/tau2.
 * For Pr <= 1 the heat flux is the quasi-conserved field (Sec. II.A.2): the
 * first stage relaxes the stresses with tau1, the second the heat flux with
 * tau2, so mu = tau1 p and kappa = C_p p tau2, Pr = tau1/tau2.  READING (the
 * paper takes the quasi-equilibria from a companion reference): f* = f^eq +
 * w_i (q_f . v_i)(|v_i|^2/(D+2) - 1), the Grad heat-flux term built from the
 * translational heat flux q_f = 1/2 sum |v-u|^2 (v-u) f (third-order Hermite
 * term: zero mass, momentum, energy and stress on the GH5 quadrature); g* =
 * g^eq + w_i (q_g . v_i), q_g = sum (v - u) g (first-order Hermite term).
 * Then f*, g* keep every conserved field and carry the heat fluxes of f, g.
 * Parity of this reading is unpinned against the paper; its transport
 * (viscosity tau1 T, diffusivity tau2 T, so Pr = tau1/tau2) and gamma are
 * pinned by the oracle tests.
 * Layout: state [2*25][n], f planes 0..24 then g planes 25..49.
 */
typedef struct {
    double rho, ux, uy, E, T, qfx, qfy, qgx, qgy;
} orc_ddf_mom;

static orc_ddf_mom ddf_moments(const orc_rule* r, const double* f, const double* g, double cv)
{
    orc_ddf_mom m = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    double jx = 0.0, jy = 0.0;
    for (int a = 0; a < 5; ++a)
        for (int b = 0; b < 5; ++b) {
            const int i = 5 * a + b;
            m.rho += f[i];
            jx += r->v[a] * f[i];
            jy += r->v[b] * f[i];
            m.E += g[i] + 0.5 * (r->v[a] * r->v[a] + r->v[b] * r->v[b]) * f[i];
        }
    m.ux = jx / m.rho;
    m.uy = jy / m.rho;
    m.T = (m.E / m.rho - 0.5 * (m.ux * m.ux + m.uy * m.uy)) / cv;
    for (int a = 0; a < 5; ++a)
        for (int b = 0; b < 5; ++b) {
            const int i = 5 * a + b;
            const double cx = r->v[a] - m.ux, cy = r->v[b] - m.uy;
            const double c2 = cx * cx + cy * cy;
            m.qfx += 0.5 * c2 * cx * f[i];
            m.qfy += 0.5 * c2 * cy * f[i];
            m.qgx += cx * g[i];
            m.qgy += cy * g[i];
        }
    return m;
}

/* equilibria and quasi-equilibria of one cell */
static void ddf_eq_qe(const orc_rule* r, const orc_ddf_mom* m, double cv, double* feq, double* geq,
                      double* fst, double* gst)
{
    const int D = 2;
    grad_hermite_feq(r, m->rho, m->ux, m->uy, m->T, feq);
    for (int a = 0; a < 5; ++a)
        for (int b = 0; b < 5; ++b) {
            const int i = 5 * a + b;
            const double w = r->w[a] * r->w[b], vx = r->v[a], vy = r->v[b];
            const double v2 = vx * vx + vy * vy;
            geq[i] = (cv - 0.5 * D) * m->T * feq[i];
            fst[i] = feq[i] + w * (m->qfx * vx + m->qfy * vy) * (v2 / (D + 2) - 1.0);
            gst[i] = geq[i] + w * (m->qgx * vx + m->qgy * vy);
        }
}

/* sensors of one cell: s[0] = |sum f ln(f/f^eq)| + |sum g ln(g/g^eq)|,
 * s[1] = sum |f^neq| + sum |g^neq|, s[2] = S_PI (f), s[3] = |sum v g^neq +
 * sum v |v|^2/2 f^neq|, s[4] = sum |f* - f^eq| + sum |g* - g^eq|
 * (eqs. HKL-sensor, sensor-neq-kin, sensor-TauNS-kin, sensor-qNSF-kin-ryk,
 * Sensor-qe-kin).  Returns 1 on a positivity fault (s[0] = +inf). */
static int ddf_sensors(const orc_rule* r, const double* f, const double* g, const double* feq,
                       const double* geq, const double* fst, const double* gst, double* s)
{
    int fault = 0;
    double klf = 0.0, klg = 0.0, neq = 0.0, pxx = 0.0, pxy = 0.0, pyy = 0.0, qx = 0.0, qy = 0.0,
           qe = 0.0;
    for (int a = 0; a < 5; ++a)
        for (int b = 0; b < 5; ++b) {
            const int i = 5 * a + b;
            const double vx = r->v[a], vy = r->v[b];
            const double fn = f[i] - feq[i], gn = g[i] - geq[i];
            if (!(f[i] > 0.0) || !(feq[i] > 0.0) || !(g[i] > 0.0) || !(geq[i] > 0.0)) {
                fault = 1;
            } else {
                klf += f[i] * log(f[i] / feq[i]);
                klg += g[i] * log(g[i] / geq[i]);
            }
            neq += fabs(fn) + fabs(gn);
            pxx += vx * vx * fn;
            pxy += vx * vy * fn;
            pyy += vy * vy * fn;
            const double e = 0.5 * (vx * vx + vy * vy);
            qx += vx * (gn + e * fn);
            qy += vy * (gn + e * fn);
            qe += fabs(fst[i] - feq[i]) + fabs(gst[i] - geq[i]);
        }
    s[0] = fault ? INFINITY : fabs(klf) + fabs(klg);
    s[1] = neq;
    s[2] = sqrt(pxx * pxx + 2.0 * pxy * pxy + pyy * pyy);
    s[3] = sqrt(qx * qx + qy * qy);
    s[4] = qe;
    return fault;
}

static uint8_t ddf_flag(const double* s, const double* thr, unsigned mask, int fault)
{
    int level = 0;
    for (int k = 0; k < 5; ++k) {
        if (!(mask & (1u << k))) continue;
        const int l = (s[k] > thr[2 * k]) + (s[k] > thr[2 * k + 1]);
        if (l > level) level = l;
    }
    if (fault) return (uint8_t)(2 | 0x80);
    return (uint8_t)level;
}

/* Extension sensors of the double distribution (the rest of Table I with
 * the g terms superposed, Sec. III; the QE collision of eq. new_collision_fi
 * as Omega): per cell, literal definitions.
 *   KN        sum |f^neq/f^eq| + sum |g^neq/g^eq|        (eqs. sensor-Knudsen-kin_f/_g)
 *   HR        |H(f) - H(f^eq)| + |H(g) - H(g^eq)|, H(h) = sum h ln(h/w)  (eq. Hneq-sensor)
 *   SIGMA_H   -(sum Omega_f ln(f/w) + sum Omega_g ln(g/w))   (eq. Dissip-H-sensor)
 *   SIGMA_HKL -(sum Omega_f ln(f/f^eq) + sum Omega_g ln(g/g^eq))  (eq. Dissip-HKL-sensor)
 *   ALPHA     |2 - alpha_f| + |2 - alpha_g|, the printed polynomial of each  (eqs. sensor-alpha-kin,
 *             alpha-polynomial-1/2)
 *   SHEAR     |(1/mu)[(tr P/D) I - P]|, P = sum v v f^neq     (eq. sensor-S-kin)
 *   QH        |u . P|                                         (eq. sensor-qH-kin)
 *   QF        |sum v g^neq + sum v |v|^2/2 f^neq - u . P|      (eq. sensor-qF-kin-ryk)
 *   COMP      sqrt(D)|tr P|/|2 mu + D lambda|                  (eq. sensor-C-kin)
 *   STRAIN    |(1/2mu)[lambda/(D eta) tr(P) I - P]|_F          (eq. sensor-E-kin)
 * with the model's second viscosity lambda = -(R/C_v) mu = -(gamma - 1) mu
 * and bulk viscosity eta = (2/D - R/C_v) mu = (2 - gamma) mu (D = 2, R = 1;
 * Sec. II.A.2, eqs. viscHeating and visc_bluk_1), the Chapman-Enskog limit
 * that compression waves on this oracle reproduce (test_oracle_ddf_ext.py).
 * Omega = -(h - h*)/tau1 - (h* - h^eq)/tau2, tau1 = mu/(rho T), tau2 = tau1/Pr.
 * A positivity fault (any of f, f^eq, g, g^eq not > 0) gives +inf for the
 * five log/ratio sensors. */
static void ddf_cell_ext(const orc_rule* r, const double* f, const double* g, double cv, double mu,
                         double prandtl, double* s)
{
    const int D = 2;
    double fe[25], ge[25], fs[25], gs[25];
    const orc_ddf_mom m = ddf_moments(r, f, g, cv);
    ddf_eq_qe(r, &m, cv, fe, ge, fs, gs);
    const double tau1 = mu / (m.rho * m.T), tau2 = tau1 / prandtl;
    double kn = 0.0, hf = 0.0, hfe = 0.0, hg = 0.0, hge = 0.0, sh = 0.0, shkl = 0.0;
    double af[5] = {0, 0, 0, 0, 0}, ag[5] = {0, 0, 0, 0, 0};
    double pxx = 0.0, pxy = 0.0, pyy = 0.0, qx = 0.0, qy = 0.0;
    int fault = 0;
    for (int a = 0; a < 5; ++a)
        for (int b = 0; b < 5; ++b) {
            const int i = 5 * a + b;
            const double vx = r->v[a], vy = r->v[b], w = r->w[a] * r->w[b];
            const double fn = f[i] - fe[i], gn = g[i] - ge[i];
            pxx += vx * vx * fn;
            pxy += vx * vy * fn;
            pyy += vy * vy * fn;
            const double e = 0.5 * (vx * vx + vy * vy);
            qx += vx * (gn + e * fn);
            qy += vy * (gn + e * fn);
            if (!(f[i] > 0.0) || !(fe[i] > 0.0) || !(g[i] > 0.0) || !(ge[i] > 0.0)) {
                fault = 1;
                continue;
            }
            const double of = -(f[i] - fs[i]) / tau1 - (fs[i] - fe[i]) / tau2;
            const double og = -(g[i] - gs[i]) / tau1 - (gs[i] - ge[i]) / tau2;
            kn += fabs(fn / fe[i]) + fabs(gn / ge[i]);
            hf += f[i] * log(f[i] / w);
            hfe += fe[i] * log(fe[i] / w);
            hg += g[i] * log(g[i] / w);
            hge += ge[i] * log(ge[i] / w);
            sh -= of * log(f[i] / w) + og * log(g[i] / w);
            shkl -= of * log(f[i] / fe[i]) + og * log(g[i] / ge[i]);
            for (int n = 1; n <= 4; ++n) {
                af[n] += pow(fn, n + 1) / pow(f[i], n);
                ag[n] += pow(gn, n + 1) / pow(g[i], n);
            }
        }
    double adev = 0.0;
    for (int k = 0; k < 2; ++k) {
        double* an = k ? ag : af;
        for (int n = 1; n <= 4; ++n) an[n] *= ((n % 2) ? 1.0 : -1.0) / (n * (n + 1.0));
        if (an[1] != 0.0) {
            const double r2 = an[2] / an[1], r3 = an[3] / an[1], r4 = an[4] / an[1];
            const double alpha = 2.0 - 4.0 * r2 + 16.0 * r2 * r2 - 8.0 * r3 + 80.0 * r2 * r3
                                 - 80.0 * r2 * r2 * r2 - 16.0 * r4;
            adev += fabs(2.0 - alpha);
        }
    }
    const double tr = pxx + pyy;
    const double sxx = (tr / D - pxx) / mu, syy = (tr / D - pyy) / mu, sxy = -pxy / mu;
    const double hx = m.ux * pxx + m.uy * pxy, hy = m.ux * pxy + m.uy * pyy;
    s[ORC_X_KN] = fault ? INFINITY : kn;
    s[ORC_X_HR] = fault ? INFINITY : fabs(hf - hfe) + fabs(hg - hge);
    s[ORC_X_SIGMA_H] = fault ? INFINITY : sh;
    s[ORC_X_SIGMA_HKL] = fault ? INFINITY : shkl;
    s[ORC_X_ALPHA] = fault ? INFINITY : adev;
    s[ORC_X_SHEAR] = sqrt(sxx * sxx + 2.0 * sxy * sxy + syy * syy);
    s[ORC_X_QH] = sqrt(hx * hx + hy * hy);
    s[ORC_X_QF] = sqrt((qx - hx) * (qx - hx) + (qy - hy) * (qy - hy));
    const double lambda = -mu / cv, eta = 2.0 * mu / D + lambda;
    s[ORC_X_COMP] = sqrt((double)D) * fabs(tr) / fabs(2.0 * mu + D * lambda);
    const double c = lambda / (D * eta);
    const double exx = (c * tr - pxx) / (2.0 * mu), eyy = (c * tr - pyy) / (2.0 * mu), exy = -pxy / (2.0 * mu);
    s[ORC_X_STRAIN] = sqrt(exx * exx + 2.0 * exy * exy + eyy * eyy);
}

/* extension sensors of n cells of a double-distribution state [50][n]:
 * out [ORC_NEXT][n] */
int orc_ddf_ext_sensors(long n, const double* f, double cv, double mu, double prandtl, double* out)
{
    orc_rule r;
    rule_d2q25(&r);
#pragma omp parallel for schedule(static)
    for (long c = 0; c < n; ++c) {
        double fc[25], gc[25], s[ORC_NEXT];
        for (int i = 0; i < 25; ++i) {
            fc[i] = f[(long)i * n + c];
            gc[i] = f[(long)(25 + i) * n + c];
        }
        ddf_cell_ext(&r, fc, gc, cv, mu, prandtl, s);
        for (int k = 0; k < ORC_NEXT; ++k) out[(long)k * n + c] = s[k];
    }
    return 0;
}

/* equilibrium (f^eq, g^eq) of n cells from FP64 fields: out [50][n] */
int orc_ddf_equilibrium(long n, const double* rho, const double* ux, const double* uy,
                        const double* T, double cv, double* out)
{
    orc_rule r;
    rule_d2q25(&r);
#pragma omp parallel for schedule(static)
    for (long c = 0; c < n; ++c) {
        double fe[25];
        grad_hermite_feq(&r, rho[c], ux[c], uy[c], T[c], fe);
        for (int i = 0; i < 25; ++i) {
            out[(long)i * n + c] = fe[i];
            out[(long)(25 + i) * n + c] = (cv - 1.0) * T[c] * fe[i];
        }
    }
    return 0;
}

/* per cell: out[0..3][n] = rho, ux, uy, T; then [4..99 +] the populations
 * feq, geq, f*, g* ([100][n] starting at plane 4) when qe != NULL */
int orc_ddf_moments(long n, const double* f, double cv, double* out, double* qe)
{
    orc_rule r;
    rule_d2q25(&r);
#pragma omp parallel for schedule(static)
    for (long c = 0; c < n; ++c) {
        double fc[25], gc[25], fe[25], ge[25], fs[25], gs[25];
        for (int i = 0; i < 25; ++i) {
            fc[i] = f[(long)i * n + c];
            gc[i] = f[(long)(25 + i) * n + c];
        }
        const orc_ddf_mom m = ddf_moments(&r, fc, gc, cv);
        out[c] = m.rho;
        out[n + c] = m.ux;
        out[2 * n + c] = m.uy;
        out[3 * n + c] = m.T;
        if (qe) {
            ddf_eq_qe(&r, &m, cv, fe, ge, fs, gs);
            for (int i = 0; i < 25; ++i) {
                qe[(long)i * n + c] = fe[i];
                qe[(long)(25 + i) * n + c] = ge[i];
                qe[(long)(50 + i) * n + c] = fs[i];
                qe[(long)(75 + i) * n + c] = gs[i];
            }
        }
    }
    return 0;
}

/* One explicit-Euler FV step of (f, g): both distributions take the same
 * dimension-by-dimension van Leer fluxes as the single-distribution step and
 * the quasi-equilibrium collision; tau1 = mu/(rho T), tau2 = tau1/Pr.
 * Sensors [5][n], flags and sums of the state the collision reads.  thr:
 * [5][2]; sums[8]: mass, x/y momentum, total energy, totals of s[0..3]. */
long orc_ddf_step(int nx, int ny, double mu, double prandtl, double cv, double dt, double dx,
                  int bc_x, int bc_y, const double* f, double* fout, double* mom, double* sens,
                  uint8_t* flags, const double* thr, unsigned mask, double* sums)
{
    orc_rule r;
    rule_d2q25(&r);
    const long n = (long)nx * ny;
    double* rowsum = (double*)calloc((size_t)ny * ORC_NSUMS, sizeof(double));
    long faults = 0;

#pragma omp parallel for schedule(static) reduction(+ : faults)
    for (int y = 0; y < ny; ++y) {
        double* rs = rowsum + (size_t)y * ORC_NSUMS;
        for (int x = 0; x < nx; ++x) {
            const long c = (long)y * nx + x;
            double fc[25], gc[25], fe[25], ge[25], fs[25], gs[25], s[5];
            for (int i = 0; i < 25; ++i) {
                fc[i] = f[(long)i * n + c];
                gc[i] = f[(long)(25 + i) * n + c];
            }
            const orc_ddf_mom m = ddf_moments(&r, fc, gc, cv);
            ddf_eq_qe(&r, &m, cv, fe, ge, fs, gs);
            const int fault = ddf_sensors(&r, fc, gc, fe, ge, fs, gs, s);
            faults += fault;
            const double tau1 = mu / (m.rho * m.T), tau2 = tau1 / prandtl;
            for (int dist = 0; dist < 2; ++dist)
                for (int a = 0; a < 5; ++a)
                    for (int b = 0; b < 5; ++b) {
                        const int i = 5 * a + b;
                        const double* fi = f + (long)(25 * dist + i) * n;
                        const double vx = r.v[a], vy = r.v[b];
                        double div = 0.0;
                        if (vx != 0.0) {
                            double q[5];
                            for (int k = -2; k <= 2; ++k)
                                q[k + 2] = fi[(long)y * nx + ghost(x + k, nx, bc_x)];
                            div += (face_flux(vx, q[1], q[2], q[3], q[4]) -
                                    face_flux(vx, q[0], q[1], q[2], q[3])) / dx;
                        }
                        if (vy != 0.0) {
                            double q[5];
                            for (int k = -2; k <= 2; ++k)
                                q[k + 2] = fi[ghost(y + k, ny, bc_y) * nx + x];
                            div += (face_flux(vy, q[1], q[2], q[3], q[4]) -
                                    face_flux(vy, q[0], q[1], q[2], q[3])) / dx;
                        }
                        const double cur = dist ? gc[i] : fc[i];
                        const double st = dist ? gs[i] : fs[i];
                        const double eq = dist ? ge[i] : fe[i];
                        const double omega = -(cur - st) / tau1 - (st - eq) / tau2;
                        fout[(long)(25 * dist + i) * n + c] = cur - dt * div + dt * omega;
                    }
            if (mom) {
                mom[c] = m.rho;
                mom[n + c] = m.ux;
                mom[2 * n + c] = m.uy;
                mom[3 * n + c] = m.T;
            }
            if (sens)
                for (int k = 0; k < 5; ++k) sens[(long)k * n + c] = s[k];
            if (flags) flags[c] = ddf_flag(s, thr, mask, fault);
            rs[0] += m.rho;
            rs[1] += m.rho * m.ux;
            rs[2] += m.rho * m.uy;
            rs[3] += m.E;
            for (int k = 0; k < 4; ++k) rs[4 + k] += s[k];
        }
    }
    for (int k = 0; k < ORC_NSUMS; ++k) sums[k] = 0.0;
    for (int y = 0; y < ny; ++y)
        for (int k = 0; k < ORC_NSUMS; ++k) sums[k] += rowsum[(size_t)y * ORC_NSUMS + k];
    free(rowsum);
    return faults;
}

/* Run nsteps of the double distribution from f ([50][n], overwritten).
 * Per step sums[step][8]; the last step's moments [4][n], sensors [5][n]
 * and flags [n] when non-NULL.  thr [5][2]. */
long orc_ddf_run(int nx, int ny, double mu, double prandtl, double cv, double dt, double dx,
                 int bc_x, int bc_y, int nsteps, double* f, double* mom, double* sens,
                 uint8_t* flags, const double* thr, unsigned mask, double* sums, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    const long n = (long)nx * ny;
    double* a = f;
    double* b = (double*)malloc(sizeof(double) * 50 * (size_t)n);
    uint8_t* fl = (uint8_t*)malloc((size_t)n);
    long faults = 0;
    for (int s = 0; s < nsteps; ++s) {
        const int last = (s == nsteps - 1);
        faults += orc_ddf_step(nx, ny, mu, prandtl, cv, dt, dx, bc_x, bc_y, a, b, last ? mom : NULL,
                               last ? sens : NULL, fl, thr, mask, sums + 8 * (long)s);
        if (last && flags) memcpy(flags, fl, (size_t)n);
        double* t = a;
        a = b;
        b = t;
    }
    if (a != f) {
        memcpy(f, a, sizeof(double) * 50 * (size_t)n);
        free(a);
    } else {
        free(b);
    }
    free(fl);
    return faults;
}

/* ------------------------------------------------------------------------ */
/* Multi-step drivers                                                        */
/* ------------------------------------------------------------------------ */

/* params for the run drivers */
typedef struct {
    int lattice, nx, ny, bc_x, bc_y;
    double tau, mu, dt, dx;
    unsigned mask;
    double thr[8];
} orc_params;

/* Run nsteps from the populations in f ([Q][n], overwritten with the final
 * post-collision state).  Per step: sums[step][8] and flag_counts[step][3]
 * (cells at level 1, level 2, and with the fault bit).  The last step's
 * moments [4][n], sensors [4][n] and flags [n] are written when non-NULL.
 * Returns the total number of fault cells over all steps. */
long orc_run(const orc_params* p, int nsteps, double* f, double* mom, double* sens,
             uint8_t* flags, double* sums, int64_t* flag_counts, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    const int Q = p->lattice;
    const long n = (long)p->nx * p->ny;
    double* a = f;
    double* b = (double*)malloc(sizeof(double) * (size_t)Q * (size_t)n);
    uint8_t* fl = (uint8_t*)malloc((size_t)n);
    long faults = 0;
    for (int s = 0; s < nsteps; ++s) {
        const int last = (s == nsteps - 1);
        if (Q == 9)
            faults += orc_d2q9_step(p->nx, p->ny, p->tau, a, b, NULL, last ? mom : NULL,
                                    last ? sens : NULL, fl, p->thr, p->mask, sums + 8 * (long)s);
        else
            faults += orc_d2q25_step(p->nx, p->ny, p->mu, p->dt, p->dx, p->bc_x, p->bc_y, a, b,
                                     last ? mom : NULL, last ? sens : NULL, fl, p->thr, p->mask,
                                     sums + 8 * (long)s);
        if (flag_counts) {
            int64_t c1 = 0, c2 = 0, cf = 0;
            for (long c = 0; c < n; ++c) {
                c1 += (fl[c] & 0x7f) == 1;
                c2 += (fl[c] & 0x7f) == 2;
                cf += (fl[c] & 0x80) != 0;
            }
            flag_counts[3 * (long)s] = c1;
            flag_counts[3 * (long)s + 1] = c2;
            flag_counts[3 * (long)s + 2] = cf;
        }
        if (last && flags) memcpy(flags, fl, (size_t)n);
        double* t = a;
        a = b;
        b = t;
    }
    if (a != f) {
        memcpy(f, a, sizeof(double) * (size_t)Q * (size_t)n);
        free(a);
    } else {
        free(b);
    }
    free(fl);
    return faults;
}

int orc_nsums(void) { return ORC_NSUMS; }
