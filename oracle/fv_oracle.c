/*
 * fv_oracle.c -- plain, slow FP64 CPU reference ("the oracle") for the explicit
 * finite-volume method of Lye, "Alsvinn: A fast multi-GPGPU finite volume solver with a
 * strong emphasis on reproducibility" (arXiv:1912.07645).
 *
 * TEST INFRASTRUCTURE ONLY. Only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark load this file. The GPU library shares no code, header, table or
 * constant with it.
 *
 * What it computes:
 *   - the conservation law u_t + div F(u) = 0 (eq. 1.1) for linear advection, Burgers and
 *     the compressible Euler equations (gamma law) in 1, 2 or 3 space dimensions, and the
 *     shallow-water equations (h, hu; flux hu u + g h^2 / 2) in 1 or 2;
 *   - its semi-discrete finite-volume form (eq. 2.1): d/dt U_i = -sum_k (F_{i+1/2 e_k} -
 *     F_{i-1/2 e_k}) / dx_k, with the numerical fluxes (Rusanov, HLL, HLLC), the
 *     reconstructions (piecewise constant, MUSCL with minmod, third-order WENO) and the SSP
 *     Runge--Kutta time steppers (forward Euler, SSP-RK2, SSP-RK3) named in Section 2.1;
 *   - a CFL time step from the maximum wave speed, and the Monte Carlo statistics named in
 *     Section 2.2 (per-cell mean and variance over samples, two-point structure functions
 *     along the axes and over cube or ball shells, point and joint PDFs), and the single-
 *     and multi-level Monte Carlo estimators of Section 2.2.
 *
 * Every pass is a separate loop over plain arrays in the order the method takes it:
 * ghost fill into a padded copy, reconstruction of the two face values of every cell,
 * numerical flux at every face, flux-difference divergence, Runge--Kutta combination.
 * Nothing is blocked, fused or reordered. Each floating-point expression is written with
 * explicit parentheses in the evaluation order of the arithmetic contract (no
 * reassociation; compile with -ffp-contract=off and without fast-math). Fused
 * multiply-adds (one rounding) appear only where written as fma(): in the WENO3 smoothness
 * terms, candidate and numerator, and in the HLLC contact-speed numerator, star energy and
 * star flux.
 *
 * Readings where the paper is silent (it names the schemes but prints no formulas):
 *   - reconstruction acts component-wise on the conserved variables;
 *   - WENO3 uses the Jiang--Shu smoothness indicators, eps = 1e-6, power 2, linear weights
 *     (2/3, 1/3), written with one division: w = (2 t1 q0 + t0 q1) / (2 t1 + t0);
 *   - HLL and HLLC take Davis wave-speed estimates SL = min(uL-cL, uR-cR),
 *     SR = max(uL+cL, uR+cR); HLLC is Toro--Spruce--Speares with the star state of
 *     Toro's book (ties: SL >= 0 takes FL, SR <= 0 takes FR, S* >= 0 takes the left star);
 *   - the SSP Runge--Kutta stages are written in increment form
 *     U^(s) = U^n + beta_s ((U^(s-1) - U^n) + dt L(U^(s-1))), beta = {1}, {1, 1/2},
 *     {1, 1/4, 2/3}, algebraically the Shu--Osher form;
 *   - dt = cfl / max_cells max_d (|u_d| + c) / dx_d, the last step clipped to end at T;
 *   - transmissive boundaries copy the edge cell into every ghost layer;
 *   - the Roe flux (Section 2.1 names it) uses Roe's average state and Harten's entropy fix
 *     on the acoustic waves (roe_euler); for Burgers the Roe speed is (uL + uR) / 2 with the
 *     fix over the rarefaction fan, for advection the velocity (plain upwinding);
 *   - Godunov's flux (Section 2.1) is the flux of the exact Riemann solution at x/t = 0, for
 *     the Euler equations by Toro's pressure-function Newton iteration (a fixed 20 steps from
 *     the primitive-variable guess) and wave sampling (godunov_euler); it calls pow(), which
 *     the device library need not round like this one, so the GPU agrees to rounding only;
 *   - the entropy-conservative fluxes Section 2.1 names: the two-point fluxes are Tadmor's
 *     (uL^2 + uL uR + uR^2) / 6 for Burgers and Chandrashekar's (logarithmic means of rho and
 *     rho / (2p)) for Euler (ec_euler); the fourth-order flux is LeFloch--Mercier--Rohde's
 *     combination of the two-point flux over the cells i-1..i+2 (ec4_face), on the cell
 *     values without reconstruction. The Euler flux calls log1p(), which the device library
 *     need not round like this one;
 *   - ENO (Section 2.1) is the second-order ENO reconstruction: the one-sided difference of
 *     smaller magnitude, the left one on a tie;
 *   - ideal MHD (the introduction names it beside Euler and shallow water as an instance of
 *     eq. 1.1; no form is given) carries
 *     (rho, m_x, m_y, m_z, E, B_x, B_y, B_z) in every dimension, magnetic pressure |B|^2 / 2,
 *     with the Rusanov and HLL fluxes on the fast magnetosonic speed; no divergence cleaning
 *     (the paper names none).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- problem description */

enum { OC_EQ_ADVECTION = 0, OC_EQ_BURGERS = 1, OC_EQ_EULER = 2, OC_EQ_SWE = 3, OC_EQ_MHD = 4 };
enum { OC_FLUX_RUSANOV = 0, OC_FLUX_HLL = 1, OC_FLUX_HLLC = 2, OC_FLUX_ROE = 3, OC_FLUX_EC = 4,
       OC_FLUX_GODUNOV = 5, OC_FLUX_EC4 = 6 };
enum { OC_REC_FIRST = 0, OC_REC_MUSCL = 1, OC_REC_WENO3 = 2, OC_REC_ENO2 = 3 };
enum { OC_INT_FE = 0, OC_INT_RK2 = 1, OC_INT_RK3 = 2 };
enum { OC_BC_PERIODIC = 0, OC_BC_TRANSMISSIVE = 1 };
enum { OC_OK = 0, OC_EINVAL = 1, OC_ENOTSUP = 2, OC_ENOMEM = 3,
       OC_ENONPHYS = 5, OC_EMAXSTEPS = 6, OC_ECFL = 7 };

#define OC_MAXF 8

typedef struct {
    int32_t dim;
    int32_t eq;
    int32_t flux;
    int32_t recon;
    int32_t integrator;
    int32_t bc[3];
    int64_t n[3];
    double lo[3];
    double hi[3];
    double gamma;
    double vel[3];
    double grav;      /* shallow water: gravitational acceleration g */
} oc_problem;

int oc_num_fields(const oc_problem* P)
{
    if (P->eq == OC_EQ_EULER) return P->dim + 2;
    if (P->eq == OC_EQ_MHD) return 8;
    if (P->eq == OC_EQ_SWE) return P->dim + 1;
    return 1;
}

static int64_t cells_of(const oc_problem* P)
{
    return P->n[0] * P->n[1] * P->n[2];
}

/* Two ghost layers on every active axis: the widest stencil (MUSCL, ENO2, WENO3) reaches two
 * cells beyond a face; piecewise-constant reconstruction uses only the first layer. */
static int ghost_width(const oc_problem* P)
{
    (void)P;
    return 2;
}

int oc_validate(const oc_problem* P)
{
    if (P->dim < 1 || P->dim > 3) return OC_EINVAL;
    for (int k = 0; k < 3; ++k) {
        if (P->n[k] < 1) return OC_EINVAL;
        if (k >= P->dim && P->n[k] != 1) return OC_EINVAL;
        if (k < P->dim && !(P->hi[k] > P->lo[k])) return OC_EINVAL;
        if (P->bc[k] != OC_BC_PERIODIC && P->bc[k] != OC_BC_TRANSMISSIVE) return OC_EINVAL;
    }
    if (P->eq < 0 || P->eq > 4) return OC_EINVAL;
    if (P->flux < 0 || P->flux > 6) return OC_EINVAL;
    if (P->recon < 0 || P->recon > 3) return OC_EINVAL;
    if (P->integrator < 0 || P->integrator > 2) return OC_EINVAL;
    if (P->flux == OC_FLUX_HLLC && P->eq != OC_EQ_EULER) return OC_ENOTSUP;
    if ((P->flux == OC_FLUX_EC || P->flux == OC_FLUX_EC4) &&
        P->eq != OC_EQ_BURGERS && P->eq != OC_EQ_EULER) return OC_ENOTSUP;
    if (P->flux == OC_FLUX_EC4 && P->recon != OC_REC_FIRST) return OC_ENOTSUP;
    if ((P->eq == OC_EQ_EULER || P->eq == OC_EQ_MHD) && !(P->gamma > 1.0)) return OC_EINVAL;
    if (P->eq == OC_EQ_MHD && P->flux != OC_FLUX_RUSANOV && P->flux != OC_FLUX_HLL)
        return OC_ENOTSUP;
    if (P->eq == OC_EQ_SWE) {
        if (!(P->grav > 0.0)) return OC_EINVAL;
        if (P->dim > 2) return OC_ENOTSUP;
        if (P->flux == OC_FLUX_GODUNOV) return OC_ENOTSUP;
    }
    return OC_OK;
}

/* dx_k^{-1}, computed as n_k / (hi_k - lo_k) */
static double inv_dx(const oc_problem* P, int k)
{
    return (double)P->n[k] / (P->hi[k] - P->lo[k]);
}

static double dmax(double a, double b) { return (a > b) ? a : b; }
static double dmin(double a, double b) { return (a < b) ? a : b; }

/* ---------------------------------------------------------------- physical fluxes */

/* Euler primitive quantities of one conserved state (rho, m_1..m_d, E). */
typedef struct {
    double ir;        /* 1 / rho */
    double u[3];      /* velocity */
    double p;         /* pressure */
    double c;         /* sound speed */
} oc_prim;

static oc_prim euler_prim(const double* U, int dim, double gamma, double gm1)
{
    oc_prim w;
    w.ir = 1.0 / U[0];
    w.u[0] = w.u[1] = w.u[2] = 0.0;
    for (int k = 0; k < dim; ++k) w.u[k] = U[1 + k] * w.ir;
    double ke = U[1] * w.u[0];
    if (dim >= 2) ke = ke + (U[2] * w.u[1]);
    if (dim >= 3) ke = ke + (U[3] * w.u[2]);
    ke = 0.5 * ke;
    w.p = gm1 * (U[dim + 1] - ke);
    w.c = sqrt((gamma * w.p) * w.ir);
    return w;
}

/* Euler flux in direction nd of the state U with primitives w. */
static void euler_flux(const double* U, const oc_prim* w, int dim, int nd, double* F)
{
    double un = w->u[nd];
    F[0] = U[1 + nd];
    for (int k = 0; k < dim; ++k) {
        if (k == nd) F[1 + k] = (U[1 + nd] * un) + w->p;
        else         F[1 + k] = U[1 + k] * un;
    }
    F[dim + 1] = (U[dim + 1] + w->p) * un;
}

/* Ideal MHD (rho, m_x, m_y, m_z, E, B_x, B_y, B_z) in units where the magnetic pressure is
 * |B|^2 / 2; three velocity and field components whatever the dimension. */
typedef struct {
    double ir;        /* 1 / rho */
    double u[3];      /* velocity */
    double pb;        /* magnetic pressure |B|^2 / 2 */
    double p;         /* gas pressure (gamma - 1)(E - rho |u|^2 / 2 - |B|^2 / 2) */
} oc_mhd;

static oc_mhd mhd_prim(const double* U, double gm1)
{
    oc_mhd w;
    w.ir = 1.0 / U[0];
    for (int k = 0; k < 3; ++k) w.u[k] = U[1 + k] * w.ir;
    const double ke = 0.5 * (((U[1] * w.u[0]) + (U[2] * w.u[1])) + (U[3] * w.u[2]));
    w.pb = 0.5 * (((U[5] * U[5]) + (U[6] * U[6])) + (U[7] * U[7]));
    w.p = gm1 * ((U[4] - ke) - w.pb);
    return w;
}

/* Fast magnetosonic speed along axis nd: c_f^2 = (a^2 + b^2 + sqrt((a^2 + b^2)^2 -
 * 4 a^2 b_n^2)) / 2 with a^2 = gamma p / rho, b^2 = |B|^2 / rho, b_n^2 = B_n^2 / rho. */
static double mhd_fast(const double* U, const oc_mhd* w, int nd, double gamma)
{
    const double a2 = (gamma * w->p) * w->ir;
    const double b2 = (2.0 * w->pb) * w->ir;
    const double bn2 = (U[5 + nd] * U[5 + nd]) * w->ir;
    const double s = a2 + b2;
    const double disc = dmax(0.0, (s * s) - ((4.0 * a2) * bn2));
    return sqrt(0.5 * (s + sqrt(disc)));
}

/* Ideal MHD flux along axis nd: mass m_n; momentum m_k u_n - B_n B_k + (p + |B|^2/2) on k = nd;
 * energy (E + p + |B|^2/2) u_n - B_n (u . B); induction u_n B_k - B_n u_k (zero for k = nd). */
static void mhd_flux(const double* U, const oc_mhd* w, int nd, double* F)
{
    const double un = w->u[nd], bn = U[5 + nd];
    const double pt = w->p + w->pb;
    const double ub = ((w->u[0] * U[5]) + (w->u[1] * U[6])) + (w->u[2] * U[7]);
    F[0] = U[1 + nd];
    for (int k = 0; k < 3; ++k) {
        const double f = (U[1 + k] * un) - (bn * U[5 + k]);
        F[1 + k] = (k == nd) ? (f + pt) : f;
        F[5 + k] = (un * U[5 + k]) - (bn * w->u[k]);
    }
    F[4] = ((U[4] + pt) * un) - (bn * ub);
}

/* ---------------------------------------------------------------- numerical fluxes */

/* Harten's entropy fix of a wave speed l with fan width d >= 0: |l| where |l| >= d, else
 * (l^2 + d^2) / (2 d). */
static double harten(double l, double d)
{
    const double al = fabs(l);
    return (al >= d) ? al : (((l * l) + (d * d)) / (2.0 * d));
}

/* Toro's pressure function f_K(p) of side K and its derivative: a shock for p > p_K,
 * a rarefaction otherwise. */
static void toro_fk(double p, double rK, double pK, double cK, double g, double* f, double* df)
{
    if (p > pK) {
        const double A = 2.0 / ((g + 1.0) * rK);
        const double B = ((g - 1.0) / (g + 1.0)) * pK;
        const double q = sqrt(A / (p + B));
        *f = (p - pK) * q;
        *df = q * (1.0 - (0.5 * ((p - pK) / (B + p))));
    } else {
        const double pr = p / pK;
        *f = ((2.0 * cK) / (g - 1.0)) * (pow(pr, (g - 1.0) / (2.0 * g)) - 1.0);
        *df = (1.0 / (rK * cK)) * pow(pr, -((g + 1.0) / (2.0 * g)));
    }
}

/* Godunov's flux for the Euler equations: the physical flux of the exact Riemann solution at
 * x/t = 0 (Toro, ch. 4). The star pressure solves f_L(p) + f_R(p) + (u_R - u_L) = 0 by 20
 * Newton steps from the primitive-variable guess, p kept at or above 1e-12 (p_L + p_R); the
 * state at x/t = 0 is sampled from the waves; tangential velocities are those of the side of
 * the contact. */
static void godunov_euler(const double* UL, const double* UR, const oc_prim* wl,
                          const oc_prim* wr, int dim, int nd, double g, double* Fh)
{
    const double rL = UL[0], rR = UR[0];
    const double uL = wl->u[nd], uR = wr->u[nd];
    const double pL = wl->p, pR = wr->p, cL = wl->c, cR = wr->c;
    const double floor_p = 1e-12 * (pL + pR);
    double p = (0.5 * (pL + pR)) - (0.125 * (((uR - uL) * (rL + rR)) * (cL + cR)));
    p = dmax(floor_p, p);
    double fL, dfL, fR, dfR;
    for (int it = 0; it < 20; ++it) {
        toro_fk(p, rL, pL, cL, g, &fL, &dfL);
        toro_fk(p, rR, pR, cR, g, &fR, &dfR);
        p = dmax(floor_p, p - (((fL + fR) + (uR - uL)) / (dfL + dfR)));
    }
    toro_fk(p, rL, pL, cL, g, &fL, &dfL);
    toro_fk(p, rR, pR, cR, g, &fR, &dfR);
    const double um = (0.5 * (uL + uR)) + (0.5 * (fR - fL));
    const double g1 = (g - 1.0) / (2.0 * g), g6 = (g - 1.0) / (g + 1.0);
    double rho, un, pr;
    const int left = (um >= 0.0);
    /* side K and its sign: the right side is the left side mirrored (u -> -u) */
    const double sg = left ? 1.0 : -1.0;
    const double rK = left ? rL : rR, pK = left ? pL : pR, cK = left ? cL : cR;
    const double uK = sg * (left ? uL : uR), umK = sg * um;
    if (p > pK) {
        const double SK = uK - (cK * sqrt((((g + 1.0) / (2.0 * g)) * (p / pK)) + g1));
        if (SK >= 0.0) { rho = rK; un = uK; pr = pK; }
        else { rho = rK * (((p / pK) + g6) / ((g6 * (p / pK)) + 1.0)); un = umK; pr = p; }
    } else if (uK - cK >= 0.0) {
        rho = rK; un = uK; pr = pK;
    } else {
        const double cm = cK * pow(p / pK, g1);
        if (umK - cm < 0.0) {
            rho = rK * pow(p / pK, 1.0 / g); un = umK; pr = p;
        } else {
            const double c = (2.0 / (g + 1.0)) * (cK + (((g - 1.0) / 2.0) * uK));
            un = c;
            rho = rK * pow(c / cK, 2.0 / (g - 1.0));
            pr = pK * pow(c / cK, (2.0 * g) / (g - 1.0));
        }
    }
    un = sg * un;
    const oc_prim* wt = left ? wl : wr;
    double u[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < dim; ++k) u[k] = (k == nd) ? un : wt->u[k];
    double ke = rho * (u[0] * u[0]);
    for (int k = 1; k < dim; ++k) ke = ke + (rho * (u[k] * u[k]));
    const double E = (pr / (g - 1.0)) + (0.5 * ke);
    Fh[0] = rho * un;
    for (int k = 0; k < dim; ++k) Fh[1 + k] = ((rho * u[k]) * un) + ((k == nd) ? pr : 0.0);
    Fh[dim + 1] = (E + pr) * un;
}

/* Logarithmic mean (a - b) / (ln a - ln b) of a, b > 0 (= a when a = b). With
 * f = (a - b) / (a + b) it equals ((a + b) / 2) f / atanh(f); for f^2 < 1e-4 the series
 * f / atanh(f) = 1 / (1 + f^2/3 + f^4/5 + f^6/7 + ...) is summed to the f^6 term (the rest is
 * below 1.2e-17 relative). Otherwise ln a - ln b = log1p((a - b) / b), whose argument carries
 * no cancellation. */
static double logmean(double a, double b)
{
    const double f = (a - b) / (a + b);
    const double u = f * f;
    if (u < 1e-4) {
        const double s = 1.0 + (u * ((1.0 / 3.0) + (u * ((1.0 / 5.0) + (u * (1.0 / 7.0))))));
        return (0.5 * (a + b)) / s;
    }
    return (a - b) / log1p((a - b) / b);
}

/* Chandrashekar's entropy-conservative (and kinetic-energy-preserving) two-point flux for
 * the Euler equations, entropy -rho s / (gamma - 1): with beta = rho / (2 p), logarithmic
 * means rho^ and beta^, arithmetic means of u_k, rho and beta, and the mean of |u|^2,
 *   F_rho = rho^ u_n, F_m_k = u_k F_rho + p~ delta_kn with p~ = mean(rho) / (2 mean(beta)),
 *   F_E = (1 / (2 (gamma - 1) beta^) - mean(|u|^2) / 2) F_rho + sum_k mean(u_k) F_m_k. */
static void ec_euler(const double* UL, const double* UR, const oc_prim* wl, const oc_prim* wr,
                     int dim, int nd, double gm1, double* Fh)
{
    const double bL = UL[0] / (2.0 * wl->p), bR = UR[0] / (2.0 * wr->p);
    const double rho_ln = logmean(UL[0], UR[0]);
    const double beta_ln = logmean(bL, bR);
    double um[3] = {0.0, 0.0, 0.0}, qL = 0.0, qR = 0.0;
    for (int k = 0; k < dim; ++k) {
        um[k] = 0.5 * (wl->u[k] + wr->u[k]);
        qL = qL + (wl->u[k] * wl->u[k]);
        qR = qR + (wr->u[k] * wr->u[k]);
    }
    const double pt = (0.5 * (UL[0] + UR[0])) / (bL + bR);
    const double Fr = rho_ln * um[nd];
    Fh[0] = Fr;
    double Fe = ((1.0 / ((2.0 * gm1) * beta_ln)) - (0.25 * (qL + qR))) * Fr;
    for (int k = 0; k < dim; ++k) {
        Fh[1 + k] = (um[k] * Fr) + ((k == nd) ? pt : 0.0);
        Fe = Fe + (um[k] * Fh[1 + k]);
    }
    Fh[dim + 1] = Fe;
}

/* Roe's flux for the Euler equations: F = (F_L + F_R)/2 - (1/2) sum_i |l_i| alpha_i K_i over
 * the eigen-decomposition of the Jacobian at Roe's average state (u~, H~ weighted by sqrt(rho);
 * a~^2 = (gamma - 1)(H~ - |u~|^2 / 2); rho~ = sqrt(rho_L rho_R)), with the wave strengths
 *   alpha_1 = (dp - rho~ a~ du_n) / (2 a~^2),  alpha_2 = d rho - dp / a~^2,
 *   alpha_3 = (dp + rho~ a~ du_n) / (2 a~^2),  beta_k = rho~ du_k (k tangential),
 * the eigenvectors K_1 = (1, u~ - a~ n, H~ - u~_n a~), K_2 = (1, u~, |u~|^2/2),
 * K_3 = (1, u~ + a~ n, H~ + u~_n a~) and the shear vectors (0, e_k, u~_k), and Harten's fix
 * on the acoustic speeds with fan widths d_1,3 = max(0, l_1,3(U_R) - l_1,3(U_L)) / 2. The
 * waves are summed in the order 1, 2, shear (k ascending), 3. */
static void roe_euler(const double* UL, const double* UR, const oc_prim* wl, const oc_prim* wr,
                      const double* FL, const double* FR, int dim, int nd, double gm1, double* Fh)
{
    const double sL = sqrt(UL[0]), sR = sqrt(UR[0]);
    const double ssum = sL + sR;
    const double HL = (UL[dim + 1] + wl->p) * wl->ir;
    const double HR = (UR[dim + 1] + wr->p) * wr->ir;
    double ut[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < dim; ++k) ut[k] = ((sL * wl->u[k]) + (sR * wr->u[k])) / ssum;
    const double Ht = ((sL * HL) + (sR * HR)) / ssum;
    double q2 = ut[0] * ut[0];
    for (int k = 1; k < dim; ++k) q2 = q2 + (ut[k] * ut[k]);
    const double a2 = gm1 * (Ht - (0.5 * q2));
    const double a = sqrt(a2);
    const double rt = sL * sR;
    const double un = ut[nd];
    const double dr = UR[0] - UL[0];
    const double dp = wr->p - wl->p;
    const double dun = wr->u[nd] - wl->u[nd];
    const double ra = rt * a;
    const double alpha1 = (dp - (ra * dun)) / (2.0 * a2);
    const double alpha2 = dr - (dp / a2);
    const double alpha3 = (dp + (ra * dun)) / (2.0 * a2);
    const double d1 = 0.5 * dmax(0.0, (wr->u[nd] - wr->c) - (wl->u[nd] - wl->c));
    const double d3 = 0.5 * dmax(0.0, (wr->u[nd] + wr->c) - (wl->u[nd] + wl->c));
    const double w1 = harten(un - a, d1) * alpha1;
    const double w2 = fabs(un) * alpha2;
    const double w3 = harten(un + a, d3) * alpha3;
    double ws[3] = {0.0, 0.0, 0.0};   /* shear waves */
    for (int k = 0; k < dim; ++k)
        if (k != nd) ws[k] = fabs(un) * (rt * (wr->u[k] - wl->u[k]));
    double D[OC_MAXF];
    D[0] = (w1 + w2) + w3;
    for (int k = 0; k < dim; ++k) {
        double t = (w1 * ((k == nd) ? (ut[k] - a) : ut[k])) + (w2 * ut[k]);
        if (k != nd) t = t + ws[k];
        D[1 + k] = t + (w3 * ((k == nd) ? (ut[k] + a) : ut[k]));
    }
    double e = (w1 * (Ht - (un * a))) + (w2 * (0.5 * q2));
    for (int k = 0; k < dim; ++k)
        if (k != nd) e = e + (ws[k] * ut[k]);
    D[dim + 1] = e + (w3 * (Ht + (un * a)));
    for (int q = 0; q < dim + 2; ++q) Fh[q] = 0.5 * ((FL[q] + FR[q]) - D[q]);
}

/* Shallow water (h, hu_1..hu_d): velocity u_k = hu_k * (1/h), celerity c = sqrt(g h), flux
 * along nd (hu_nd, hu_k u_nd + (k == nd) g h^2 / 2). */
typedef struct {
    double ih;        /* 1 / h */
    double u[2];
    double c;
} oc_swe;

static oc_swe swe_prim(const double* U, int dim, double g)
{
    oc_swe w;
    w.ih = 1.0 / U[0];
    w.u[0] = w.u[1] = 0.0;
    for (int k = 0; k < dim; ++k) w.u[k] = U[1 + k] * w.ih;
    w.c = sqrt(g * U[0]);
    return w;
}

static void swe_flux(const double* U, const oc_swe* w, int dim, int nd, double g, double* F)
{
    const double un = w->u[nd];
    const double hp = 0.5 * (g * (U[0] * U[0]));
    F[0] = U[1 + nd];
    for (int k = 0; k < dim; ++k) F[1 + k] = (k == nd) ? ((U[1 + k] * un) + hp) : (U[1 + k] * un);
}

/* Roe's flux for shallow water: average velocity weighted by sqrt(h), celerity
 * c~ = sqrt(g (h_L + h_R) / 2), strengths alpha_1,2 = (dh -+ (d(hu_n) - u~_n dh) / c~) / 2
 * on the fields u~_n -+ c~ with eigenvectors (1, u~ -+ c~ n), shear strengths
 * d(hu_k) - u~_k dh on the fields u~_n with eigenvectors (0, e_k); Harten's fix on the two
 * gravity waves with fan widths max(0, l(U_R) - l(U_L)) / 2; fields summed in the order
 * u - c, shear (k ascending), u + c. */
static void roe_swe(const double* UL, const double* UR, const oc_swe* wl, const oc_swe* wr,
                    const double* FL, const double* FR, int dim, int nd, double g, double* Fh)
{
    const double sL = sqrt(UL[0]), sR = sqrt(UR[0]);
    const double ssum = sL + sR;
    double ut[2] = {0.0, 0.0};
    for (int k = 0; k < dim; ++k) ut[k] = ((sL * wl->u[k]) + (sR * wr->u[k])) / ssum;
    const double ct = sqrt(g * (0.5 * (UL[0] + UR[0])));
    const double un = ut[nd];
    const double dh = UR[0] - UL[0];
    const double dq = (UR[1 + nd] - UL[1 + nd]) - (un * dh);
    const double alpha1 = 0.5 * (dh - (dq / ct));
    const double alpha2 = 0.5 * (dh + (dq / ct));
    const double d1 = 0.5 * dmax(0.0, (wr->u[nd] - wr->c) - (wl->u[nd] - wl->c));
    const double d2 = 0.5 * dmax(0.0, (wr->u[nd] + wr->c) - (wl->u[nd] + wl->c));
    const double w1 = harten(un - ct, d1) * alpha1;
    const double w2 = harten(un + ct, d2) * alpha2;
    double D[OC_MAXF];
    D[0] = w1 + w2;
    for (int k = 0; k < dim; ++k) {
        double t = w1 * ((k == nd) ? (un - ct) : ut[k]);
        if (k != nd) t = t + (fabs(un) * ((UR[1 + k] - UL[1 + k]) - (ut[k] * dh)));
        D[1 + k] = t + (w2 * ((k == nd) ? (un + ct) : ut[k]));
    }
    for (int q = 0; q < dim + 1; ++q) Fh[q] = 0.5 * ((FL[q] + FR[q]) - D[q]);
}

/* Numerical flux across a face with normal direction nd, from the reconstructed states
 * UL (left of the face) and UR (right of the face). */
void oc_numerical_flux(const oc_problem* P, int nd, const double* UL, const double* UR,
                       double* Fh)
{
    const int nf = oc_num_fields(P);
    if (P->eq == OC_EQ_MHD) {
        const double gm1 = P->gamma - 1.0;
        oc_mhd wl = mhd_prim(UL, gm1);
        oc_mhd wr = mhd_prim(UR, gm1);
        double FL[OC_MAXF], FR[OC_MAXF];
        mhd_flux(UL, &wl, nd, FL);
        mhd_flux(UR, &wr, nd, FR);
        const double uL = wl.u[nd], uR = wr.u[nd];
        const double cL = mhd_fast(UL, &wl, nd, P->gamma), cR = mhd_fast(UR, &wr, nd, P->gamma);
        if (P->flux == OC_FLUX_RUSANOV) {
            double s = dmax(fabs(uL) + cL, fabs(uR) + cR);
            for (int q = 0; q < nf; ++q)
                Fh[q] = 0.5 * ((FL[q] + FR[q]) - (s * (UR[q] - UL[q])));
            return;
        }
        double SL = dmin(uL - cL, uR - cR);
        double SR = dmax(uL + cL, uR + cR);
        if (SL >= 0.0) { for (int q = 0; q < nf; ++q) Fh[q] = FL[q]; return; }
        if (SR <= 0.0) { for (int q = 0; q < nf; ++q) Fh[q] = FR[q]; return; }
        for (int q = 0; q < nf; ++q)
            Fh[q] = (((SR * FL[q]) - (SL * FR[q])) + ((SL * SR) * (UR[q] - UL[q]))) / (SR - SL);
        return;
    }
    if (P->eq == OC_EQ_SWE) {
        const int dim = P->dim;
        const double g = P->grav;
        oc_swe wl = swe_prim(UL, dim, g);
        oc_swe wr = swe_prim(UR, dim, g);
        double FL[OC_MAXF], FR[OC_MAXF];
        swe_flux(UL, &wl, dim, nd, g, FL);
        swe_flux(UR, &wr, dim, nd, g, FR);
        const double uL = wl.u[nd], uR = wr.u[nd];
        if (P->flux == OC_FLUX_RUSANOV) {
            double s = dmax(fabs(uL) + wl.c, fabs(uR) + wr.c);
            for (int q = 0; q < nf; ++q)
                Fh[q] = 0.5 * ((FL[q] + FR[q]) - (s * (UR[q] - UL[q])));
            return;
        }
        if (P->flux == OC_FLUX_ROE) {
            roe_swe(UL, UR, &wl, &wr, FL, FR, dim, nd, g, Fh);
            return;
        }
        double SL = dmin(uL - wl.c, uR - wr.c);
        double SR = dmax(uL + wl.c, uR + wr.c);
        if (SL >= 0.0) { for (int q = 0; q < nf; ++q) Fh[q] = FL[q]; return; }
        if (SR <= 0.0) { for (int q = 0; q < nf; ++q) Fh[q] = FR[q]; return; }
        for (int q = 0; q < nf; ++q)
            Fh[q] = (((SR * FL[q]) - (SL * FR[q])) + ((SL * SR) * (UR[q] - UL[q]))) / (SR - SL);
        return;
    }
    if (P->eq == OC_EQ_EULER) {
        const int dim = P->dim;
        const double gamma = P->gamma;
        const double gm1 = gamma - 1.0;
        oc_prim wl = euler_prim(UL, dim, gamma, gm1);
        oc_prim wr = euler_prim(UR, dim, gamma, gm1);
        double FL[OC_MAXF], FR[OC_MAXF];
        euler_flux(UL, &wl, dim, nd, FL);
        euler_flux(UR, &wr, dim, nd, FR);
        const double uL = wl.u[nd], uR = wr.u[nd];
        if (P->flux == OC_FLUX_RUSANOV) {
            double s = dmax(fabs(uL) + wl.c, fabs(uR) + wr.c);
            for (int q = 0; q < nf; ++q)
                Fh[q] = 0.5 * ((FL[q] + FR[q]) - (s * (UR[q] - UL[q])));
            return;
        }
        if (P->flux == OC_FLUX_ROE) {
            roe_euler(UL, UR, &wl, &wr, FL, FR, dim, nd, gm1, Fh);
            return;
        }
        if (P->flux == OC_FLUX_GODUNOV) {
            godunov_euler(UL, UR, &wl, &wr, dim, nd, gamma, Fh);
            return;
        }
        if (P->flux == OC_FLUX_EC || P->flux == OC_FLUX_EC4) {
            ec_euler(UL, UR, &wl, &wr, dim, nd, gm1, Fh);
            return;
        }
        double SL = dmin(uL - wl.c, uR - wr.c);
        double SR = dmax(uL + wl.c, uR + wr.c);
        if (SL >= 0.0) { for (int q = 0; q < nf; ++q) Fh[q] = FL[q]; return; }
        if (SR <= 0.0) { for (int q = 0; q < nf; ++q) Fh[q] = FR[q]; return; }
        if (P->flux == OC_FLUX_HLL) {
            for (int q = 0; q < nf; ++q)
                Fh[q] = (((SR * FL[q]) - (SL * FR[q])) + ((SL * SR) * (UR[q] - UL[q])))
                        / (SR - SL);
            return;
        }
        /* HLLC: contact speed S* and the star state on the side it selects. */
        double DL = UL[0] * (SL - uL);
        double DR = UR[0] * (SR - uR);
        double num = (wr.p - wl.p) + fma(UL[1 + nd], SL - uL, -(UR[1 + nd] * (SR - uR)));
        double den = DL - DR;
        double Ss = num / den;
        const double* UK; const double* FK; const oc_prim* wK; double SK, DK;
        if (Ss >= 0.0) { UK = UL; FK = FL; wK = &wl; SK = SL; DK = DL; }
        else           { UK = UR; FK = FR; wK = &wr; SK = SR; DK = DR; }
        double uK = wK->u[nd];
        double f = DK / (SK - Ss);
        double Us[OC_MAXF];
        Us[0] = f;
        for (int k = 0; k < dim; ++k)
            Us[1 + k] = (k == nd) ? (f * Ss) : (f * wK->u[k]);
        Us[dim + 1] = f * fma(UK[dim + 1], wK->ir, (Ss - uK) * (Ss + (wK->p / DK)));
        for (int q = 0; q < nf; ++q)
            Fh[q] = fma(SK, Us[q] - UK[q], FK[q]);
        return;
    }
    /* scalar equations */
    double uL = UL[0], uR = UR[0];
    double FL, FR, s, SL, SR;
    if (P->eq == OC_EQ_BURGERS) {
        FL = 0.5 * (uL * uL);
        FR = 0.5 * (uR * uR);
        s = dmax(fabs(uL), fabs(uR));
        SL = dmin(uL, uR);
        SR = dmax(uL, uR);
    } else {
        double a = P->vel[nd];
        FL = a * uL;
        FR = a * uR;
        s = fabs(a);
        SL = a;
        SR = a;
    }
    if (P->flux == OC_FLUX_RUSANOV) {
        Fh[0] = 0.5 * ((FL + FR) - (s * (uR - uL)));
        return;
    }
    if (P->flux == OC_FLUX_ROE) {
        /* Roe speed: the mean for Burgers (the exact Rankine--Hugoniot speed), the velocity for
         * advection; Harten's fix over the fan width of a Burgers rarefaction */
        double a, d;
        if (P->eq == OC_EQ_BURGERS) {
            a = 0.5 * (uL + uR);
            d = 0.5 * dmax(0.0, uR - uL);
        } else {
            a = P->vel[nd];
            d = 0.0;
        }
        Fh[0] = 0.5 * ((FL + FR) - (harten(a, d) * (uR - uL)));
        return;
    }
    if (P->flux == OC_FLUX_GODUNOV) {
        /* the exact Riemann solution at x/t = 0: for Burgers the shock speed (uL + uR)/2 picks
         * the side, a transonic rarefaction gives f(0) = 0; advection is upwinding */
        if (P->eq == OC_EQ_BURGERS) {
            if (uL > uR) {
                Fh[0] = ((0.5 * (uL + uR)) >= 0.0) ? FL : FR;
            } else {
                Fh[0] = (uL >= 0.0) ? FL : ((uR <= 0.0) ? FR : 0.0);
            }
        } else {
            Fh[0] = (P->vel[nd] >= 0.0) ? FL : FR;
        }
        return;
    }
    if (P->flux == OC_FLUX_EC || P->flux == OC_FLUX_EC4) {
        /* Tadmor's entropy-conservative flux for Burgers (entropy u^2 / 2) */
        Fh[0] = (((uL * uL) + (uL * uR)) + (uR * uR)) / 6.0;
        return;
    }
    if (SL >= 0.0) { Fh[0] = FL; return; }
    if (SR <= 0.0) { Fh[0] = FR; return; }
    Fh[0] = (((SR * FL) - (SL * FR)) + ((SL * SR) * (uR - uL))) / (SR - SL);
}

/* ---------------------------------------------------------------- reconstruction */

/* minmod of two one-sided differences (sign tests, no product). */
static double minmod(double a, double b)
{
    if (a > 0.0 && b > 0.0) return dmin(a, b);
    if (a < 0.0 && b < 0.0) return dmax(a, b);
    return 0.0;
}

/* Third-order WENO value at the face between b and c, from the cells (a, b, c):
 * candidates q0 = (b + c)/2 on {b, c} and q1 = (3b - a)/2 on {a, b}, smoothness
 * beta0 = (c-b)^2, beta1 = (b-a)^2, linear weights 2/3 and 1/3, eps = 1e-6, power 2. */
double oc_weno3(double a, double b, double c)
{
    const double eps = 1e-6;
    double d0 = b - a;
    double d1 = c - b;
    double t0 = fma(d1, d1, eps);
    t0 = t0 * t0;
    double t1 = fma(d0, d0, eps);
    t1 = t1 * t1;
    double q0 = 0.5 * (b + c);
    double q1 = fma(1.5, b, -(0.5 * a));
    return fma(2.0 * t1, q0, t0 * q1) / ((2.0 * t1) + t0);
}

/* Face values of the cell with stencil values (um, u0, up) = (U_{i-1}, U_i, U_{i+1}):
 * *minus = value at i-1/2, *plus = value at i+1/2. */
static void reconstruct(int recon, double um, double u0, double up, double* minus, double* plus)
{
    if (recon == OC_REC_FIRST) {
        *minus = u0;
        *plus = u0;
    } else if (recon == OC_REC_MUSCL) {
        double sigma = minmod(u0 - um, up - u0);
        *plus = u0 + (0.5 * sigma);
        *minus = u0 - (0.5 * sigma);
    } else if (recon == OC_REC_ENO2) {
        /* second-order ENO: the one-sided difference of smaller magnitude (left on a tie) */
        double dl = u0 - um, dr = up - u0;
        double sigma = (fabs(dl) <= fabs(dr)) ? dl : dr;
        *plus = u0 + (0.5 * sigma);
        *minus = u0 - (0.5 * sigma);
    } else {
        *plus = oc_weno3(um, u0, up);
        *minus = oc_weno3(up, u0, um);
    }
}

/* The face values (i - 1/2, i + 1/2) of one cell, for the pins. */
void oc_reconstruct(int recon, double um, double u0, double up, double* minus, double* plus)
{
    reconstruct(recon, um, u0, up, minus, plus);
}

/* ---------------------------------------------------------------- one right-hand side */

static int64_t map_index(int64_t i, int64_t n, int bc)
{
    if (bc == OC_BC_PERIODIC) {
        int64_t r = i % n;
        return r < 0 ? r + n : r;
    }
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

/* Padded extents: g ghost layers on each side of every active axis. */
typedef struct {
    int64_t m[3];     /* padded sizes */
    int g[3];         /* ghost width per axis (0 on inactive axes) */
} oc_pad;

static oc_pad pad_of(const oc_problem* P)
{
    oc_pad pd;
    int g = ghost_width(P);
    for (int k = 0; k < 3; ++k) {
        pd.g[k] = (k < P->dim) ? g : 0;
        pd.m[k] = P->n[k] + 2 * pd.g[k];
    }
    return pd;
}

static int64_t pidx(const oc_pad* pd, int64_t i, int64_t j, int64_t k)
{
    return ((k + pd->g[2]) * pd->m[1] + (j + pd->g[1])) * pd->m[0] + (i + pd->g[0]);
}

/* Step 1: ghost-cell fill. Copy one sample U[f][cells] into padded arrays, filling each
 * ghost cell from the interior cell that the boundary condition maps it to. */
static void ghost_fill(const oc_problem* P, const oc_pad* pd, const double* U, double* W)
{
    const int nf = oc_num_fields(P);
    const int64_t N = cells_of(P);
    const int64_t PN = pd->m[0] * pd->m[1] * pd->m[2];
    for (int f = 0; f < nf; ++f) {
        #pragma omp parallel for collapse(2) schedule(static)
        for (int64_t kk = 0; kk < pd->m[2]; ++kk)
            for (int64_t jj = 0; jj < pd->m[1]; ++jj)
                for (int64_t ii = 0; ii < pd->m[0]; ++ii) {
                    int64_t i = map_index(ii - pd->g[0], P->n[0], P->bc[0]);
                    int64_t j = map_index(jj - pd->g[1], P->n[1], P->bc[1]);
                    int64_t k = map_index(kk - pd->g[2], P->n[2], P->bc[2]);
                    W[f * PN + (kk * pd->m[1] + jj) * pd->m[0] + ii] =
                        U[f * N + (k * P->n[1] + j) * P->n[0] + i];
                }
    }
}

/* L(U) = -sum_k (F_{i+1/2 e_k} - F_{i-1/2 e_k}) / dx_k for one sample (eq. 2.1). */
/* Fourth-order entropy-conservative flux of LeFloch, Mercier and Rohde at the face between
 * cells i = cL and i + 1 of the padded array W: the combination
 *   F = sum_{r=1,2} alpha_r sum_{s=0}^{r-1} F~(U_{i-s}, U_{i-s+r}),  alpha = (4/3, -1/6),
 * of the two-point entropy-conservative flux F~, i.e.
 *   F = (4/3) F~(U_i, U_{i+1}) - (1/6) (F~(U_i, U_{i+2}) + F~(U_{i-1}, U_{i+1})).
 * It acts on the cell values themselves (no reconstruction). */
static void ec4_face(const oc_problem* P, int d, const double* W, int64_t PN, int64_t cL,
                     int64_t stride, double* F)
{
    const int nf = oc_num_fields(P);
    double A[OC_MAXF], B[OC_MAXF], C[OC_MAXF], D[OC_MAXF];
    double F1[OC_MAXF], F2[OC_MAXF], F3[OC_MAXF];
    for (int f = 0; f < nf; ++f) {
        A[f] = W[f * PN + cL - stride];
        B[f] = W[f * PN + cL];
        C[f] = W[f * PN + cL + stride];
        D[f] = W[f * PN + cL + 2 * stride];
    }
    oc_numerical_flux(P, d, B, C, F1);
    oc_numerical_flux(P, d, B, D, F2);
    oc_numerical_flux(P, d, A, C, F3);
    for (int f = 0; f < nf; ++f)
        F[f] = ((4.0 / 3.0) * F1[f]) - ((1.0 / 6.0) * (F2[f] + F3[f]));
}

int oc_rhs(const oc_problem* P, const double* U, double* rhs)
{
    int st = oc_validate(P);
    if (st) return st;
    const int nf = oc_num_fields(P);
    const int dim = P->dim;
    const int64_t N = cells_of(P);
    const int64_t nx = P->n[0], ny = P->n[1], nz = P->n[2];
    oc_pad pd = pad_of(P);
    const int64_t PN = pd.m[0] * pd.m[1] * pd.m[2];

    double* W = (double*)malloc(sizeof(double) * (size_t)(PN * nf));
    /* face values of every cell (incl. one ghost layer) along the current direction */
    double* Wm = (double*)malloc(sizeof(double) * (size_t)(PN * nf));
    double* Wp = (double*)malloc(sizeof(double) * (size_t)(PN * nf));
    /* fluxes at the n_d + 1 faces along the current direction, interior elsewhere */
    int64_t nface_max = (nx + 1) * ny * nz;
    if (dim >= 2 && nx * (ny + 1) * nz > nface_max) nface_max = nx * (ny + 1) * nz;
    if (dim >= 3 && nx * ny * (nz + 1) > nface_max) nface_max = nx * ny * (nz + 1);
    double* Fh = (double*)malloc(sizeof(double) * (size_t)(nface_max * nf));
    /* accumulated flux differences, per field and cell */
    double* acc = (double*)malloc(sizeof(double) * (size_t)(N * nf));
    if (!W || !Wm || !Wp || !Fh || !acc) {
        free(W); free(Wm); free(Wp); free(Fh); free(acc);
        return OC_ENOMEM;
    }

    ghost_fill(P, &pd, U, W);

    for (int d = 0; d < dim; ++d) {
        const int64_t e[3] = { d == 0, d == 1, d == 2 };
        const int64_t stride = (d == 0) ? 1 : (d == 1 ? pd.m[0] : pd.m[0] * pd.m[1]);
        /* Step 2: reconstruction. Face values of every cell in the range [-1, n_d] along d
         * (interior along the other axes). */
        for (int f = 0; f < nf; ++f) {
            const double* Wf = W + f * PN;
            #pragma omp parallel for collapse(2) schedule(static)
            for (int64_t k = -e[2]; k < nz + e[2]; ++k)
                for (int64_t j = -e[1]; j < ny + e[1]; ++j)
                    for (int64_t i = -e[0]; i < nx + e[0]; ++i) {
                        int64_t c = pidx(&pd, i, j, k);
                        reconstruct(P->recon, Wf[c - stride], Wf[c], Wf[c + stride],
                                    &Wm[f * PN + c], &Wp[f * PN + c]);
                    }
        }
        /* Step 3: numerical flux at every face along d. Face index (i, j, k) along d is the
         * face between cell idx - e_d and cell idx. */
        const int64_t fx = nx + e[0], fy = ny + e[1], fz = nz + e[2];
        const int64_t NF = fx * fy * fz;
        const double a_inv = inv_dx(P, d);
        #pragma omp parallel for collapse(2) schedule(static)
        for (int64_t k = 0; k < fz; ++k)
            for (int64_t j = 0; j < fy; ++j)
                for (int64_t i = 0; i < fx; ++i) {
                    int64_t cR = pidx(&pd, i, j, k);
                    int64_t cL = cR - stride;
                    double UL[OC_MAXF], UR[OC_MAXF], F[OC_MAXF];
                    if (P->flux == OC_FLUX_EC4) {
                        ec4_face(P, d, W, PN, cL, stride, F);
                    } else {
                        for (int f = 0; f < nf; ++f) {
                            UL[f] = Wp[f * PN + cL];
                            UR[f] = Wm[f * PN + cR];
                        }
                        oc_numerical_flux(P, d, UL, UR, F);
                    }
                    int64_t fi = (k * fy + j) * fx + i;
                    for (int f = 0; f < nf; ++f) Fh[f * NF + fi] = F[f];
                }
        /* Step 4: flux difference along d, added in direction order x, y, z. */
        #pragma omp parallel for collapse(2) schedule(static)
        for (int64_t k = 0; k < nz; ++k)
            for (int64_t j = 0; j < ny; ++j)
                for (int64_t i = 0; i < nx; ++i) {
                    int64_t fm = (k * fy + j) * fx + i;
                    int64_t fp = ((k + e[2]) * fy + (j + e[1])) * fx + (i + e[0]);
                    int64_t cell = (k * ny + j) * nx + i;
                    for (int f = 0; f < nf; ++f) {
                        double term = (Fh[f * NF + fp] - Fh[f * NF + fm]) * a_inv;
                        if (d == 0) acc[f * N + cell] = term;
                        else        acc[f * N + cell] = acc[f * N + cell] + term;
                    }
                }
    }
    #pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < N * nf; ++c) rhs[c] = -acc[c];

    free(W); free(Wm); free(Wp); free(Fh); free(acc);
    return OC_OK;
}

/* ---------------------------------------------------------------- wave speed / CFL */

/* Maximum over cells and directions of (|u_d| + c) / dx_d for one sample, and whether any
 * cell is non-physical (rho <= 0, p <= 0, h <= 0 or a non-finite component). */
void oc_max_speed(const oc_problem* P, const double* U, double* M_out, int* bad_out)
{
    const int nf = oc_num_fields(P);
    const int64_t N = cells_of(P);
    const int dim = P->dim;
    const double gamma = P->gamma, gm1 = P->gamma - 1.0;
    double M = 0.0;
    int bad = 0;
    for (int64_t c = 0; c < N; ++c) {
        double V[OC_MAXF];
        for (int f = 0; f < nf; ++f) {
            V[f] = U[f * N + c];
            if (!isfinite(V[f])) bad = 1;
        }
        double m = 0.0;
        if (P->eq == OC_EQ_EULER) {
            oc_prim w = euler_prim(V, dim, gamma, gm1);
            if (!(V[0] > 0.0) || !(w.p > 0.0)) bad = 1;
            for (int d = 0; d < dim; ++d) {
                double a = (fabs(w.u[d]) + w.c) * inv_dx(P, d);
                m = (d == 0) ? a : dmax(m, a);
            }
        } else if (P->eq == OC_EQ_MHD) {
            oc_mhd w = mhd_prim(V, gm1);
            if (!(V[0] > 0.0) || !(w.p > 0.0)) bad = 1;
            for (int d = 0; d < dim; ++d) {
                double a = (fabs(w.u[d]) + mhd_fast(V, &w, d, gamma)) * inv_dx(P, d);
                m = (d == 0) ? a : dmax(m, a);
            }
        } else if (P->eq == OC_EQ_SWE) {
            oc_swe w = swe_prim(V, dim, P->grav);
            if (!(V[0] > 0.0)) bad = 1;
            for (int d = 0; d < dim; ++d) {
                double a = (fabs(w.u[d]) + w.c) * inv_dx(P, d);
                m = (d == 0) ? a : dmax(m, a);
            }
        } else {
            for (int d = 0; d < dim; ++d) {
                double s = (P->eq == OC_EQ_BURGERS) ? fabs(V[0]) : fabs(P->vel[d]);
                double a = s * inv_dx(P, d);
                m = (d == 0) ? a : dmax(m, a);
            }
        }
        if (m > M) M = m;
    }
    *M_out = M;
    *bad_out = bad;
}

/* ---------------------------------------------------------------- time stepping */

static int n_stages(int integrator)
{
    return integrator == OC_INT_FE ? 1 : (integrator == OC_INT_RK2 ? 2 : 3);
}

static double stage_beta(int integrator, int s)
{
    if (s == 0) return 1.0;
    if (integrator == OC_INT_RK2) return 0.5;
    return (s == 1) ? 0.25 : (2.0 / 3.0);
}

/* One full SSP Runge--Kutta step of size dt on one sample, in place. */
int oc_step(const oc_problem* P, double* U, double dt)
{
    const int nf = oc_num_fields(P);
    const int64_t N = cells_of(P) * nf;
    double* Un = (double*)malloc(sizeof(double) * (size_t)N);
    double* Us = (double*)malloc(sizeof(double) * (size_t)N);
    double* R = (double*)malloc(sizeof(double) * (size_t)N);
    if (!Un || !Us || !R) { free(Un); free(Us); free(R); return OC_ENOMEM; }
    memcpy(Un, U, sizeof(double) * (size_t)N);
    memcpy(Us, U, sizeof(double) * (size_t)N);
    const int S = n_stages(P->integrator);
    int st = OC_OK;
    for (int s = 0; s < S && st == OC_OK; ++s) {
        st = oc_rhs(P, Us, R);
        const double beta = stage_beta(P->integrator, s);
        #pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < N; ++c)
            Us[c] = Un[c] + (beta * ((Us[c] - Un[c]) + (dt * R[c])));
    }
    if (st == OC_OK) memcpy(U, Us, sizeof(double) * (size_t)N);
    free(Un); free(Us); free(R);
    return st;
}

/* Evolve each sample of U[batch][fields][cells] from t[b] to t_end with adaptive CFL
 * steps. Per sample: steps[b] = number of steps taken, err[b] = status. The state is
 * checked (non-physical values) before every step and at the end. */
int oc_evolve(const oc_problem* P, double* U, int64_t batch, double* t, double t_end,
              double cfl, int64_t max_steps, int64_t* steps, int32_t* err)
{
    int st = oc_validate(P);
    if (st) return st;
    if (!(cfl > 0.0) || cfl > 1.0 || batch < 0 || max_steps < 0) return OC_EINVAL;
    const int nf = oc_num_fields(P);
    const int64_t N = cells_of(P) * nf;
    int rc = OC_OK;
    for (int64_t b = 0; b < batch; ++b) {
        double* Ub = U + b * N;
        double tb = t[b];
        int64_t k = 0;
        int32_t e = OC_OK;
        for (;;) {
            double M;
            int bad;
            oc_max_speed(P, Ub, &M, &bad);
            if (bad) { e = OC_ENONPHYS; break; }
            if (!(tb < t_end)) break;
            if (k >= max_steps) { e = OC_EMAXSTEPS; break; }
            double dt = (M == 0.0) ? (t_end - tb) : (cfl / M);
            int last = 0;
            if (tb + dt >= t_end) { dt = t_end - tb; last = 1; }
            int s2 = oc_step(P, Ub, dt);
            if (s2) return s2;
            tb = last ? t_end : (tb + dt);
            k += 1;
        }
        t[b] = tb;
        if (steps) steps[b] = k;
        if (err) err[b] = e;
        if (e != OC_OK && rc == OC_OK) rc = e;
    }
    return rc;
}

/* Fixed time step: nsteps steps of size dt for every sample. Fails a sample with
 * OC_ECFL when dt * M exceeds cfl_bound before a step, OC_ENONPHYS on a bad state. */
int oc_evolve_fixed_dt(const oc_problem* P, double* U, int64_t batch, double dt,
                       int64_t nsteps, double cfl_bound, int32_t* err)
{
    int st = oc_validate(P);
    if (st) return st;
    if (!(dt > 0.0) || nsteps < 0 || batch < 0) return OC_EINVAL;
    const int nf = oc_num_fields(P);
    const int64_t N = cells_of(P) * nf;
    int rc = OC_OK;
    for (int64_t b = 0; b < batch; ++b) {
        double* Ub = U + b * N;
        int32_t e = OC_OK;
        for (int64_t k = 0; k <= nsteps; ++k) {
            double M;
            int bad;
            oc_max_speed(P, Ub, &M, &bad);
            if (bad) { e = OC_ENONPHYS; break; }
            if (k == nsteps) break;
            if (dt * M > cfl_bound) { e = OC_ECFL; break; }
            int s2 = oc_step(P, Ub, dt);
            if (s2) return s2;
        }
        if (err) err[b] = e;
        if (e != OC_OK && rc == OC_OK) rc = e;
    }
    return rc;
}

/* ---------------------------------------------------------------- statistics */

/* Number of statistical quantities: Euler (rho, u_1..u_d, E), scalar (u). */
int oc_num_quantities(const oc_problem* P)
{
    return oc_num_fields(P);
}

/* q[quantity][cells] of one sample: rho, u_k = m_k * (1/rho), E; shallow water h,
 * u_k = hu_k * (1/h); MHD rho, u_x, u_y, u_z, E, B_x, B_y, B_z; or the scalar itself. */
void oc_quantities(const oc_problem* P, const double* U, double* q)
{
    const int nf = oc_num_fields(P);
    const int64_t N = cells_of(P);
    if (P->eq == OC_EQ_MHD) {
        for (int64_t c = 0; c < N; ++c) {
            double ir = 1.0 / U[c];
            for (int f = 0; f < 8; ++f)
                q[f * N + c] = (f >= 1 && f <= 3) ? (U[f * N + c] * ir) : U[f * N + c];
        }
        return;
    }
    if (P->eq == OC_EQ_SWE) {
        for (int64_t c = 0; c < N; ++c) {
            double ih = 1.0 / U[c];
            q[c] = U[c];
            for (int k = 0; k < P->dim; ++k) q[(1 + k) * N + c] = U[(1 + k) * N + c] * ih;
        }
        return;
    }
    if (P->eq != OC_EQ_EULER) {
        memcpy(q, U, sizeof(double) * (size_t)N);
        return;
    }
    for (int64_t c = 0; c < N; ++c) {
        double ir = 1.0 / U[c];
        q[c] = U[c];
        for (int k = 0; k < P->dim; ++k) q[(1 + k) * N + c] = U[(1 + k) * N + c] * ir;
        q[(nf - 1) * N + c] = U[(nf - 1) * N + c];
    }
}

/* Second-order structure function of one periodic field q[cells] at lag h (cells):
 * S(h) = (1 / (d N)) sum_{axes e} sum_x (q(x + h e) - q(x))^2, summed axis by axis in
 * row-major cell order. */
double oc_structure_function(const oc_problem* P, const double* q, int64_t h)
{
    const int64_t nx = P->n[0], ny = P->n[1], nz = P->n[2];
    double s = 0.0;
    for (int d = 0; d < P->dim; ++d) {
        for (int64_t k = 0; k < nz; ++k)
            for (int64_t j = 0; j < ny; ++j)
                for (int64_t i = 0; i < nx; ++i) {
                    int64_t i2 = (d == 0) ? (i + h) % nx : i;
                    int64_t j2 = (d == 1) ? (j + h) % ny : j;
                    int64_t k2 = (d == 2) ? (k + h) % nz : k;
                    double diff = q[(k2 * ny + j2) * nx + i2] - q[(k * ny + j) * nx + i];
                    s = s + (diff * diff);
                }
    }
    return s / ((double)P->dim * (double)cells_of(P));
}

/* Welford's update of running mean and M2 with one more observation x (n = new count). */
static void welford(double x, int64_t n, double* mean, double* m2)
{
    double delta = x - *mean;
    *mean = *mean + (delta / (double)n);
    *m2 = *m2 + (delta * (x - *mean));
}

/* Add the samples U[batch] in index order to the running statistics:
 *   mean[q][cells], m2[q][cells]    per-cell moments of the quantities;
 *   s2mean[q][max_h], s2m2[q][max_h] moments over samples of S_q(h), h = 1..max_h;
 *   *count                          number of samples seen so far (updated). */
int oc_stats_accumulate(const oc_problem* P, const double* U, int64_t batch, int32_t max_h,
                        double* mean, double* m2, double* s2mean, double* s2m2, int64_t* count)
{
    int st = oc_validate(P);
    if (st) return st;
    if (max_h > 0) {
        for (int k = 0; k < P->dim; ++k)
            if (P->bc[k] != OC_BC_PERIODIC || max_h >= P->n[k]) return OC_ENOTSUP;
    }
    const int nf = oc_num_fields(P);
    const int nq = oc_num_quantities(P);
    const int64_t N = cells_of(P);
    double* q = (double*)malloc(sizeof(double) * (size_t)(N * nq));
    if (!q) return OC_ENOMEM;
    for (int64_t b = 0; b < batch; ++b) {
        oc_quantities(P, U + b * N * nf, q);
        int64_t n = *count + 1;
        #pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < N * nq; ++c) welford(q[c], n, &mean[c], &m2[c]);
        for (int qi = 0; qi < nq; ++qi)
            for (int32_t h = 1; h <= max_h; ++h) {
                double s = oc_structure_function(P, q + qi * N, h);
                welford(s, n, &s2mean[qi * max_h + (h - 1)], &s2m2[qi * max_h + (h - 1)]);
            }
        *count = n;
    }
    free(q);
    return OC_OK;
}

/* ---------------------------------------------------------------- PDFs, shell structure functions
 *
 * Section 2.2 lists point PDFs, joint PDFs and two-point structure functions among the
 * statistics (after Fjordholm, Lye and Mishra) and prints no formula for them. Readings:
 *   - point PDF: the histogram over samples of one quantity at one cell. nbins equal bins
 *     on [lo, hi): bin k = floor(((v - lo) / (hi - lo)) * nbins), taken as nbins - 1 if
 *     rounding gives nbins; one more counter for values below lo and one for values not
 *     below hi (NaN included), so the counters of a point add up to the number of samples;
 *   - joint PDF: the histogram over samples of the pair (quantity a at cell x, quantity b at
 *     cell y) on nbins x nbins such bins, plus one counter for pairs with either value
 *     outside its range;
 *   - shell structure function of order p in {1, 2} at radius h on the periodic grid:
 *     S_p(h) = 1/(N |A_h|) sum_{o in A_h} sum_x |q(x + o) - q(x)|^p, where A_h is the cube
 *     shell {o in Z^d : max_k |o_k| = h} or the ball shell {o : (h-1)^2 < |o|^2 <= h^2}.
 *     Offsets are taken with o_z, o_y, o_x ascending, cells in row-major order.
 */

/* Bin of v: 0..nbins-1, -1 below lo, nbins not below hi. */
static int pdf_bin(double v, double lo, double hi, int32_t nbins)
{
    if (v < lo) return -1;
    if (!(v < hi)) return nbins;
    const int64_t k = (int64_t)floor(((v - lo) / (hi - lo)) * (double)nbins);
    return (int)(k < nbins ? k : nbins - 1);
}

/* Quantity qi of one sample U[fields][cells] at cell c (as oc_quantities computes it). */
static double cell_quantity(const oc_problem* P, const double* U, int64_t c, int qi)
{
    const int64_t N = cells_of(P);
    if (P->eq == OC_EQ_SWE && qi > 0) {
        double ih = 1.0 / U[c];
        return U[qi * N + c] * ih;
    }
    if (P->eq == OC_EQ_MHD) {
        if (qi < 1 || qi > 3) return U[qi * N + c];
        double ir = 1.0 / U[c];
        return U[qi * N + c] * ir;
    }
    if (P->eq != OC_EQ_EULER || qi == 0 || qi == oc_num_fields(P) - 1) return U[qi * N + c];
    double ir = 1.0 / U[c];
    return U[qi * N + c] * ir;
}

static int pdf_args_ok(const oc_problem* P, int32_t quantity, double lo, double hi, int32_t nbins)
{
    return quantity >= 0 && quantity < oc_num_quantities(P) && nbins >= 1 && lo < hi;
}

/* Point PDFs of quantity at cells points[npoints] over the samples U[batch], added to
 * counts[npoints][nbins + 2] (bins, then below, then above). */
int oc_point_pdf(const oc_problem* P, const double* U, int64_t batch, int32_t quantity,
                 int64_t npoints, const int64_t* points, double lo, double hi, int32_t nbins,
                 int64_t* counts)
{
    int st = oc_validate(P);
    if (st) return st;
    const int64_t N = cells_of(P);
    if (!pdf_args_ok(P, quantity, lo, hi, nbins) || batch < 0 || npoints < 0) return OC_EINVAL;
    for (int64_t i = 0; i < npoints; ++i)
        if (points[i] < 0 || points[i] >= N) return OC_EINVAL;
    const int nf = oc_num_fields(P);
    for (int64_t b = 0; b < batch; ++b)
        for (int64_t i = 0; i < npoints; ++i) {
            const int k = pdf_bin(cell_quantity(P, U + b * nf * N, points[i], quantity), lo, hi, nbins);
            const int slot = (k < 0) ? nbins : (k >= nbins ? nbins + 1 : k);
            counts[i * (nbins + 2) + slot] += 1;
        }
    return OC_OK;
}

/* Joint PDFs of (quantity_a at pairs[i][0], quantity_b at pairs[i][1]) over the samples,
 * added to counts[npairs][nbins * nbins + 1] (bin ka * nbins + kb, then outside). */
int oc_joint_pdf(const oc_problem* P, const double* U, int64_t batch, int32_t quantity_a,
                 int32_t quantity_b, int64_t npairs, const int64_t* pairs, double lo_a,
                 double hi_a, double lo_b, double hi_b, int32_t nbins, int64_t* counts)
{
    int st = oc_validate(P);
    if (st) return st;
    const int64_t N = cells_of(P);
    if (!pdf_args_ok(P, quantity_a, lo_a, hi_a, nbins) || !pdf_args_ok(P, quantity_b, lo_b, hi_b, nbins) ||
        batch < 0 || npairs < 0)
        return OC_EINVAL;
    for (int64_t i = 0; i < 2 * npairs; ++i)
        if (pairs[i] < 0 || pairs[i] >= N) return OC_EINVAL;
    const int nf = oc_num_fields(P);
    const int64_t per = (int64_t)nbins * nbins + 1;
    for (int64_t b = 0; b < batch; ++b)
        for (int64_t i = 0; i < npairs; ++i) {
            const double* Ub = U + b * nf * N;
            const int ka = pdf_bin(cell_quantity(P, Ub, pairs[2 * i], quantity_a), lo_a, hi_a, nbins);
            const int kb = pdf_bin(cell_quantity(P, Ub, pairs[2 * i + 1], quantity_b), lo_b, hi_b, nbins);
            const int64_t slot = (ka < 0 || ka >= nbins || kb < 0 || kb >= nbins)
                                     ? per - 1 : (int64_t)ka * nbins + kb;
            counts[i * per + slot] += 1;
        }
    return OC_OK;
}

static int64_t wrap64(int64_t i, int64_t n)
{
    i %= n;
    return i < 0 ? i + n : i;
}

/* Is o in the shell A_h (cube or ball)? */
static int in_shell(int64_t ox, int64_t oy, int64_t oz, int64_t h, int ball)
{
    if (ball) {
        const int64_t r2 = ox * ox + oy * oy + oz * oz;
        return (h - 1) * (h - 1) < r2 && r2 <= h * h;
    }
    int64_t m = ox < 0 ? -ox : ox;
    const int64_t ay = oy < 0 ? -oy : oy, az = oz < 0 ? -oz : oz;
    if (ay > m) m = ay;
    if (az > m) m = az;
    return m == h;
}

/* S_p(h) of one periodic field q[cells] over the cube (ball = 0) or ball (ball = 1) shell. */
double oc_structure_shell(const oc_problem* P, const double* q, int64_t h, int32_t p, int32_t ball)
{
    const int64_t nx = P->n[0], ny = P->n[1], nz = P->n[2];
    const int64_t hy = (P->dim >= 2) ? h : 0, hz = (P->dim >= 3) ? h : 0;
    double s = 0.0;
    int64_t shell = 0;
    for (int64_t oz = -hz; oz <= hz; ++oz)
        for (int64_t oy = -hy; oy <= hy; ++oy)
            for (int64_t ox = -h; ox <= h; ++ox) {
                if (!in_shell(ox, oy, oz, h, ball)) continue;
                shell += 1;
                for (int64_t k = 0; k < nz; ++k)
                    for (int64_t j = 0; j < ny; ++j)
                        for (int64_t i = 0; i < nx; ++i) {
                            const int64_t c2 = (wrap64(k + oz, nz) * ny + wrap64(j + oy, ny)) * nx + wrap64(i + ox, nx);
                            const double d = q[c2] - q[(k * ny + j) * nx + i];
                            s = s + ((p == 1) ? fabs(d) : (d * d));
                        }
            }
    return s / ((double)cells_of(P) * (double)shell);
}

/* Shell structure functions of every quantity of every sample: out[batch][quantities][max_h]
 * with out[b][q][h - 1] = S_p(h) of quantity q of sample b. Periodic grids only, with
 * max_h < n on every active axis (OC_ENOTSUP otherwise). */
int oc_structure_shell_batch(const oc_problem* P, const double* U, int64_t batch, int32_t max_h,
                             int32_t p, int32_t ball, double* out)
{
    int st = oc_validate(P);
    if (st) return st;
    if (max_h < 1 || (p != 1 && p != 2) || (ball != 0 && ball != 1) || batch < 0) return OC_EINVAL;
    for (int k = 0; k < P->dim; ++k)
        if (P->bc[k] != OC_BC_PERIODIC || max_h >= P->n[k]) return OC_ENOTSUP;
    const int nf = oc_num_fields(P);
    const int nq = oc_num_quantities(P);
    const int64_t N = cells_of(P);
    double* q = (double*)malloc(sizeof(double) * (size_t)(N * nq));
    if (!q) return OC_ENOMEM;
    for (int64_t b = 0; b < batch; ++b) {
        oc_quantities(P, U + b * N * nf, q);
        #pragma omp parallel for schedule(dynamic) collapse(2)
        for (int qi = 0; qi < nq; ++qi)
            for (int32_t h = 1; h <= max_h; ++h)
                out[(b * nq + qi) * max_h + (h - 1)] = oc_structure_shell(P, q + qi * N, h, p, ball);
    }
    free(q);
    return OC_OK;
}

/* ---------------------------------------------------------------- multilevel Monte Carlo */

/* Integer refinement ratio of a fine grid over a coarse grid on every axis (0 if not an
 * integer ratio >= 1 on every active axis). */
static int refinement(const oc_problem* F, const oc_problem* Cp, int64_t r[3])
{
    if (F->dim != Cp->dim || oc_num_fields(F) != oc_num_fields(Cp)) return 0;
    for (int k = 0; k < 3; ++k) {
        if (Cp->n[k] < 1 || F->n[k] % Cp->n[k] != 0) return 0;
        r[k] = F->n[k] / Cp->n[k];
    }
    return 1;
}

/* Index of the coarse cell that contains fine cell (i, j, k) (piecewise-constant
 * prolongation P: every fine cell takes the value of its parent). */
static int64_t parent_cell(const oc_problem* Cp, const int64_t r[3], int64_t i, int64_t j,
                           int64_t k)
{
    return ((k / r[2]) * Cp->n[1] + (j / r[1])) * Cp->n[0] + (i / r[0]);
}

/* Level-difference statistics of the multilevel estimator (Section 2.2): for coupled
 * samples b (the same random input on the fine and the coarse grid), the per-cell running
 * moments of x = q(u_fine) - P q(u_coarse), samples added in index order. mean and m2 live on
 * the fine grid: [quantity][fine cells]. */
int oc_stats_accumulate_diff(const oc_problem* F, const oc_problem* Cp, const double* Uf,
                             const double* Uc, int64_t batch, double* mean, double* m2,
                             int64_t* count)
{
    int st = oc_validate(F);
    if (st) return st;
    st = oc_validate(Cp);
    if (st) return st;
    int64_t r[3];
    if (!refinement(F, Cp, r)) return OC_EINVAL;
    const int nf = oc_num_fields(F);
    const int64_t Nf = cells_of(F), Nc = cells_of(Cp);
    double* qf = (double*)malloc(sizeof(double) * (size_t)(Nf * nf));
    double* qc = (double*)malloc(sizeof(double) * (size_t)(Nc * nf));
    if (!qf || !qc) { free(qf); free(qc); return OC_ENOMEM; }
    for (int64_t b = 0; b < batch; ++b) {
        oc_quantities(F, Uf + b * Nf * nf, qf);
        oc_quantities(Cp, Uc + b * Nc * nf, qc);
        const int64_t n = *count + 1;
        for (int q = 0; q < nf; ++q)
            for (int64_t k = 0; k < F->n[2]; ++k)
                for (int64_t j = 0; j < F->n[1]; ++j)
                    for (int64_t i = 0; i < F->n[0]; ++i) {
                        const int64_t c = (k * F->n[1] + j) * F->n[0] + i;
                        const double x = qf[q * Nf + c] - qc[q * Nc + parent_cell(Cp, r, i, j, k)];
                        welford(x, n, &mean[q * Nf + c], &m2[q * Nf + c]);
                    }
        *count = n;
    }
    free(qf);
    free(qc);
    return OC_OK;
}

/* Multilevel estimate on the finest grid: out = sum_{l = 1..L} P_{l -> L} mean_l, levels added
 * in order (level 1 holds the plain mean, since u^0 = 0). probs[l], means[l] = [quantity][cells
 * of level l]; the last level is the finest. */
int oc_mlmc_combine(int32_t nlevels, const oc_problem* probs, const double* const* means,
                    double* out)
{
    if (nlevels < 1) return OC_EINVAL;
    const oc_problem* Fp = &probs[nlevels - 1];
    const int nf = oc_num_fields(Fp);
    const int64_t Nf = cells_of(Fp);
    for (int l = 0; l < nlevels; ++l) {
        int64_t r[3];
        if (!refinement(Fp, &probs[l], r)) return OC_EINVAL;
        const int64_t Nl = cells_of(&probs[l]);
        for (int q = 0; q < nf; ++q)
            for (int64_t k = 0; k < Fp->n[2]; ++k)
                for (int64_t j = 0; j < Fp->n[1]; ++j)
                    for (int64_t i = 0; i < Fp->n[0]; ++i) {
                        const int64_t c = (k * Fp->n[1] + j) * Fp->n[0] + i;
                        const double v = means[l][q * Nl + parent_cell(&probs[l], r, i, j, k)];
                        out[q * Nf + c] = (l == 0) ? v : (out[q * Nf + c] + v);
                    }
    }
    return OC_OK;
}

/* ---------------------------------------------------------------- misc */

int oc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
