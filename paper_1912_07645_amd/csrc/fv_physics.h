// fv_physics.h -- device functions of the finite-volume scheme (Section 2.1): physical
// fluxes, numerical fluxes at a face, face reconstruction and the wave speed.
//
// Arithmetic contract (shared, independently written, by the CPU reference used in tests):
// IEEE binary64, every expression evaluated exactly as parenthesised, no FMA contraction
// (the library is compiled with -ffp-contract=off), correctly rounded division and square
// root, min/max written as comparisons. With this the kernels reproduce the reference bit
// for bit, which a chaotic flow such as the Kelvin--Helmholtz shear layer (Section 3)
// requires for agreement at the 1e-12 level.
#pragma once

#include "fv_common.h"

namespace fvk {

template <int DIM, int EQ>
struct NumFields {
    static constexpr int value =
        (EQ == EQ_EULER) ? DIM + 2 : ((EQ == EQ_SWE) ? DIM + 1 : ((EQ == EQ_MHD) ? 8 : 1));
};

__device__ __forceinline__ double vmax(double a, double b) { return (a > b) ? a : b; }
__device__ __forceinline__ double vmin(double a, double b) { return (a < b) ? a : b; }

// ---------------------------------------------------------------- Euler (gamma law)

template <int DIM>
struct EulerPrim {
    double ir;       // 1 / rho
    double u[DIM];   // velocity m_k * ir
    double p;        // (gamma - 1) (E - ke), ke = 0.5 * sum_k m_k u_k
    double c;        // sqrt(gamma p ir)
};

template <int DIM>
__device__ __forceinline__ EulerPrim<DIM> euler_prim(const double* U, const Phys& ph)
{
    EulerPrim<DIM> w;
    w.ir = 1.0 / U[0];
#pragma unroll
    for (int k = 0; k < DIM; ++k) w.u[k] = U[1 + k] * w.ir;
    double ke = U[1] * w.u[0];
    if (DIM >= 2) ke = ke + (U[2] * w.u[1 < DIM ? 1 : 0]);
    if (DIM >= 3) ke = ke + (U[3] * w.u[2 < DIM ? 2 : 0]);
    ke = 0.5 * ke;
    w.p = ph.gm1 * (U[DIM + 1] - ke);
    w.c = sqrt((ph.gamma * w.p) * w.ir);
    return w;
}

// Select component d (0..DIM-1) of a small array; an exact copy, no arithmetic.
template <int DIM>
__device__ __forceinline__ double pick(const double* v, int d)
{
    double r = v[0];
    if (DIM >= 2) r = (d == 1) ? v[1 < DIM ? 1 : 0] : r;
    if (DIM >= 3) r = (d == 2) ? v[2 < DIM ? 2 : 0] : r;
    return r;
}

// Physical Euler flux along axis nd (run-time axis; primitives in the grid frame).
template <int DIM>
__device__ __forceinline__ void euler_flux(const double* U, const EulerPrim<DIM>& w, int nd, double* F)
{
    const double un = pick<DIM>(w.u, nd);
    F[0] = pick<DIM>(U + 1, nd);
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        const double a = U[1 + k] * un;
        F[1 + k] = (k == nd) ? (a + w.p) : a;
    }
    F[DIM + 1] = (U[DIM + 1] + w.p) * un;
}

// Harten's entropy fix of a wave speed l with fan width d >= 0.
__device__ __forceinline__ double harten_fix(double l, double d)
{
    const double al = fabs(l);
    return (al >= d) ? al : (((l * l) + (d * d)) / (2.0 * d));
}

// Roe's flux: half the sum of the two physical fluxes minus half the sum over the
// characteristic fields of the Roe-average Jacobian, |speed| x strength x eigenvector, taken
// in the order acoustic (u - a), entropy (u), shear (tangential axes ascending), acoustic
// (u + a). Average state: velocity and total enthalpy weighted by sqrt(rho), sound speed from
// (gamma - 1)(H - |u|^2 / 2), density sqrt(rho_L rho_R). Harten's fix acts on the acoustic
// speeds with half the jump of the one-sided characteristic speeds as fan width.
template <int DIM>
__device__ __forceinline__ void roe_flux(const double* UL, const double* UR, const EulerPrim<DIM>& wl,
                                         const EulerPrim<DIM>& wr, const double* FL, const double* FR,
                                         int nd, double* Fh, const Phys& ph)
{
    const double sqL = sqrt(UL[0]);
    const double sqR = sqrt(UR[0]);
    const double wsum = sqL + sqR;
    const double hL = (UL[DIM + 1] + wl.p) * wl.ir;
    const double hR = (UR[DIM + 1] + wr.p) * wr.ir;
    double ua[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) ua[k] = ((sqL * wl.u[k]) + (sqR * wr.u[k])) / wsum;
    const double ha = ((sqL * hL) + (sqR * hR)) / wsum;
    double usq = ua[0] * ua[0];
#pragma unroll
    for (int k = 1; k < DIM; ++k) usq = usq + (ua[k] * ua[k]);
    const double csq = ph.gm1 * (ha - (0.5 * usq));
    const double ca = sqrt(csq);
    const double rhoa = sqL * sqR;
    const double una = pick<DIM>(ua, nd);
    const double unL = pick<DIM>(wl.u, nd), unR = pick<DIM>(wr.u, nd);
    const double jr = UR[0] - UL[0];
    const double jp = wr.p - wl.p;
    const double jun = unR - unL;
    const double rc = rhoa * ca;
    const double s1 = (jp - (rc * jun)) / (2.0 * csq);    // strengths
    const double s2 = jr - (jp / csq);
    const double s3 = (jp + (rc * jun)) / (2.0 * csq);
    const double fan1 = 0.5 * vmax(0.0, (unR - wr.c) - (unL - wl.c));
    const double fan3 = 0.5 * vmax(0.0, (unR + wr.c) - (unL + wl.c));
    const double g1 = harten_fix(una - ca, fan1) * s1;    // |speed| x strength
    const double g2 = fabs(una) * s2;
    const double g3 = harten_fix(una + ca, fan3) * s3;
    double gs[DIM];                                        // shear fields
#pragma unroll
    for (int k = 0; k < DIM; ++k) gs[k] = fabs(una) * (rhoa * (wr.u[k] - wl.u[k]));
    double diss[DIM + 2];
    diss[0] = (g1 + g2) + g3;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        const bool n = (k == nd);
        double t = (g1 * (n ? (ua[k] - ca) : ua[k])) + (g2 * ua[k]);
        t = n ? t : (t + gs[k]);
        diss[1 + k] = t + (g3 * (n ? (ua[k] + ca) : ua[k]));
    }
    double te = (g1 * (ha - (una * ca))) + (g2 * (0.5 * usq));
#pragma unroll
    for (int k = 0; k < DIM; ++k) te = (k == nd) ? te : (te + (gs[k] * ua[k]));
    diss[DIM + 1] = te + (g3 * (ha + (una * ca)));
#pragma unroll
    for (int q = 0; q < DIM + 2; ++q) Fh[q] = 0.5 * ((FL[q] + FR[q]) - diss[q]);
}

// One side K of the exact Riemann problem: the constants of Toro's pressure function f_K(p)
// (shock branch above p_K, rarefaction branch at or below) that do not depend on p.
struct ToroSide {
    double pK, A, B, kr, idr;    // A = 2/((g+1) rho_K), B = (g-1)/(g+1) p_K, kr = 2 c_K/(g-1),
                                 // idr = 1/(rho_K c_K)
};

__device__ __forceinline__ ToroSide toro_side(double rK, double pK, double cK, double g)
{
    ToroSide s;
    s.pK = pK;
    s.A = 2.0 / ((g + 1.0) * rK);
    s.B = ((g - 1.0) / (g + 1.0)) * pK;
    s.kr = (2.0 * cK) / (g - 1.0);
    s.idr = 1.0 / (rK * cK);
    return s;
}

// (p/p_K)^e for p/p_K > 0, as exp(e ln(p/p_K)): within a few ulp for the ratios that occur
// here, and cheaper than the general pow().
__device__ __forceinline__ double ratio_pow(double pr, double e) { return exp(e * log(pr)); }

// f_K(p) and its derivative. On the rarefaction branch one power t = (p/p_K)^((g-1)/(2g))
// serves both, since (p/p_K)^(-(g+1)/(2g)) = t / (p/p_K); t is returned (negative on the
// shock branch) for the wave sampling.
__device__ __forceinline__ void toro_f(const ToroSide& s, double p, double e1, double& f, double& df,
                                       double& t)
{
    if (p > s.pK) {
        const double q = sqrt(s.A / (p + s.B));
        f = (p - s.pK) * q;
        df = q * (1.0 - (0.5 * ((p - s.pK) / (s.B + p))));
        t = -1.0;
    } else {
        const double pr = p / s.pK;
        t = ratio_pow(pr, e1);
        f = s.kr * (t - 1.0);
        df = s.idr * (t / pr);
    }
}

// Godunov's flux: the physical flux of the exact Riemann solution at x/t = 0. The star
// pressure is the root of f_L(p) + f_R(p) + (u_R - u_L), found by Newton's method from the
// primitive-variable guess, kept at or above 1e-12 (p_L + p_R) and stopped once a step moves p
// by at most 1e-8 p, or after 20 steps. Newton's error after a step of size d is about
// |f''/(2 f')| d^2, and |f''/f'| p stays below 1 on both branches of f_K (about
// (1 - (gamma-1)/(2 gamma)) / p on the rarefaction branch), so the new iterate is within
// 1e-16 p of the root. f_K(p) and t_K(p) then follow from their values at the previous iterate
// by one linear step, with a neglected term of the same size. The side of the contact that
// x/t = 0 lies on
// supplies the tangential velocities; its wave (shock or rarefaction fan) decides between the
// side's own state, the star state and the fan state. The right side is handled as the left
// side of the mirrored problem (u -> -u).
template <int DIM>
__device__ __forceinline__ void godunov_flux(const double* UL, const double* UR, const EulerPrim<DIM>& wl,
                                             const EulerPrim<DIM>& wr, int nd, double* Fh, const Phys& ph)
{
    const double g = ph.gamma;
    const double e1 = (g - 1.0) / (2.0 * g);
    const double uL = pick<DIM>(wl.u, nd), uR = pick<DIM>(wr.u, nd);
    const double du = uR - uL;
    const ToroSide sL = toro_side(UL[0], wl.p, wl.c, g);
    const ToroSide sR = toro_side(UR[0], wr.p, wr.c, g);
    const double floor_p = 1e-12 * (wl.p + wr.p);
    double p = (0.5 * (wl.p + wr.p)) - (0.125 * ((du * (UL[0] + UR[0])) * (wl.c + wr.c)));
    p = vmax(floor_p, p);
    double fL, dfL, tL, fR, dfR, tR, pold = p;
    for (int it = 0; it < 20; ++it) {
        toro_f(sL, p, e1, fL, dfL, tL);
        toro_f(sR, p, e1, fR, dfR, tR);
        pold = p;
        p = vmax(floor_p, p - (((fL + fR) + du) / (dfL + dfR)));
        if (fabs(p - pold) <= (1e-8 * pold)) break;
    }
    const double dp = p - pold;
    fL = fL + (dfL * dp);
    fR = fR + (dfR * dp);
    const double um = (0.5 * (uL + uR)) + (0.5 * (fR - fL));
    const bool left = (um >= 0.0);
    const double sg = left ? 1.0 : -1.0;
    const double rK = left ? UL[0] : UR[0];
    const double pK = left ? wl.p : wr.p;
    const double cK = left ? wl.c : wr.c;
    const double uK = sg * (left ? uL : uR);
    const double umK = sg * um;
    const double pr = p / pK;
    double rho, un, pres;
    if (p > pK) {
        const double g6 = (g - 1.0) / (g + 1.0);
        const double SK = uK - (cK * sqrt((((g + 1.0) / (2.0 * g)) * pr) + e1));
        const bool pre = (SK >= 0.0);
        rho = pre ? rK : (rK * ((pr + g6) / ((g6 * pr) + 1.0)));
        un = pre ? uK : umK;
        pres = pre ? pK : p;
    } else if (uK - cK >= 0.0) {
        rho = rK;
        un = uK;
        pres = pK;
    } else {
        // t = (p/p_K)^e1 at the root; (p/p_K)^(1/g) = (p/p_K) / t^2 since 1/g = 1 - 2 e1
        double t = left ? tL : tR;
        t = (t < 0.0) ? ratio_pow(pr, e1) : (t * (1.0 + (e1 * (dp / pold))));
        const double cm = cK * t;
        if (umK - cm < 0.0) {
            rho = rK * (pr / (t * t));
            un = umK;
            pres = p;
        } else {
            // inside the fan: c = u at x/t = 0; (c/c_K)^(2g/(g-1)) = (c/c_K)^(2/(g-1)) (c/c_K)^2
            const double c = (2.0 / (g + 1.0)) * (cK + (((g - 1.0) / 2.0) * uK));
            const double cr = c / cK;
            const double w = ratio_pow(cr, 2.0 / (g - 1.0));
            un = c;
            rho = rK * w;
            pres = pK * (w * (cr * cr));
        }
    }
    un = sg * un;
    double u[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) u[k] = (k == nd) ? un : (left ? wl.u[k] : wr.u[k]);
    double ke = rho * (u[0] * u[0]);
#pragma unroll
    for (int k = 1; k < DIM; ++k) ke = ke + (rho * (u[k] * u[k]));
    const double E = (pres / (g - 1.0)) + (0.5 * ke);
    Fh[0] = rho * un;
#pragma unroll
    for (int k = 0; k < DIM; ++k) Fh[1 + k] = ((rho * u[k]) * un) + ((k == nd) ? pres : 0.0);
    Fh[DIM + 1] = (E + pres) * un;
}

// Logarithmic mean (a - b) / (ln a - ln b) of a, b > 0 (= a when a = b). With
// f = (a - b) / (a + b) it is ((a + b) / 2) f / atanh(f); for f^2 < 1e-4 the series
// f / atanh(f) = 1 / (1 + f^2/3 + f^4/5 + f^6/7 + ...) to the f^6 term (the rest is below
// 1.2e-17 relative), otherwise ln a - ln b = log1p((a - b) / b), free of cancellation.
__device__ __forceinline__ double logmean(double a, double b)
{
    const double f = (a - b) / (a + b);
    const double u = f * f;
    if (u < 1e-4) {
        const double s = 1.0 + (u * ((1.0 / 3.0) + (u * ((1.0 / 5.0) + (u * (1.0 / 7.0))))));
        return (0.5 * (a + b)) / s;
    }
    return (a - b) / log1p((a - b) / b);
}

// Chandrashekar's entropy-conservative two-point flux (entropy -rho s / (gamma - 1)): with
// beta = rho / (2p), logarithmic means of rho and beta, arithmetic means of u_k, rho, beta
// and |u|^2: F_rho = rho^ u_n, F_m_k = u_k F_rho + p~ delta_kn, p~ = mean rho / (2 mean beta),
// F_E = (1 / (2 (gamma - 1) beta^) - mean |u|^2 / 2) F_rho + sum_k u_k F_m_k.
// beta = rho / (2 p) of a state with primitives w.
template <int DIM>
__device__ __forceinline__ double ec_beta(const double* U, const EulerPrim<DIM>& w)
{
    return U[0] / (2.0 * w.p);
}

template <int DIM>
__device__ __forceinline__ void ec_euler_flux(const double* UL, const double* UR, const EulerPrim<DIM>& wl,
                                              const EulerPrim<DIM>& wr, double bL, double bR, int nd,
                                              double* Fh, const Phys& ph)
{
    const double rho_ln = logmean(UL[0], UR[0]);
    const double beta_ln = logmean(bL, bR);
    double um[DIM];
    double qL = wl.u[0] * wl.u[0], qR = wr.u[0] * wr.u[0];
#pragma unroll
    for (int k = 0; k < DIM; ++k) um[k] = 0.5 * (wl.u[k] + wr.u[k]);
#pragma unroll
    for (int k = 1; k < DIM; ++k) {
        qL = qL + (wl.u[k] * wl.u[k]);
        qR = qR + (wr.u[k] * wr.u[k]);
    }
    const double pt = (0.5 * (UL[0] + UR[0])) / (bL + bR);
    const double Fr = rho_ln * pick<DIM>(um, nd);
    Fh[0] = Fr;
    double Fe = ((1.0 / ((2.0 * ph.gm1) * beta_ln)) - (0.25 * (qL + qR))) * Fr;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        Fh[1 + k] = (um[k] * Fr) + ((k == nd) ? pt : 0.0);
        Fe = Fe + (um[k] * Fh[1 + k]);
    }
    Fh[DIM + 1] = Fe;
}

// Numerical flux of the Euler equations across a face with normal axis nd.
template <int DIM, int FLUX>
__device__ __forceinline__ void euler_numflux(const double* UL, const double* UR, int nd, double* Fh,
                                              const Phys& ph)
{
    constexpr int NF = DIM + 2;
    const EulerPrim<DIM> wl = euler_prim<DIM>(UL, ph);
    const EulerPrim<DIM> wr = euler_prim<DIM>(UR, ph);
    double FL[NF], FR[NF];
    euler_flux<DIM>(UL, wl, nd, FL);
    euler_flux<DIM>(UR, wr, nd, FR);
    const double uL = pick<DIM>(wl.u, nd), uR = pick<DIM>(wr.u, nd);
    if (FLUX == FLUX_RUSANOV) {
        // local Lax--Friedrichs: central flux plus max-speed dissipation
        const double s = vmax(fabs(uL) + wl.c, fabs(uR) + wr.c);
#pragma unroll
        for (int q = 0; q < NF; ++q) Fh[q] = 0.5 * ((FL[q] + FR[q]) - (s * (UR[q] - UL[q])));
        return;
    }
    if (FLUX == FLUX_ROE) {
        roe_flux<DIM>(UL, UR, wl, wr, FL, FR, nd, Fh, ph);
        return;
    }
    if (FLUX == FLUX_GODUNOV) {
        godunov_flux<DIM>(UL, UR, wl, wr, nd, Fh, ph);
        return;
    }
    if (FLUX == FLUX_EC || FLUX == FLUX_EC4) {
        ec_euler_flux<DIM>(UL, UR, wl, wr, ec_beta<DIM>(UL, wl), ec_beta<DIM>(UR, wr), nd, Fh, ph);
        return;
    }
    // Davis wave-speed estimates
    const double SL = vmin(uL - wl.c, uR - wr.c);
    const double SR = vmax(uL + wl.c, uR + wr.c);
    const bool takeL = (SL >= 0.0);
    const bool takeR = (SR <= 0.0);
    if (FLUX == FLUX_HLL) {
        const double den = SR - SL;
        const double slsr = SL * SR;
#pragma unroll
        for (int q = 0; q < NF; ++q) {
            const double mid = (((SR * FL[q]) - (SL * FR[q])) + (slsr * (UR[q] - UL[q]))) / den;
            Fh[q] = takeL ? FL[q] : (takeR ? FR[q] : mid);
        }
        return;
    }
    // HLLC: contact speed, then the star state of the side it selects (one star state)
    const double mL = pick<DIM>(UL + 1, nd), mR = pick<DIM>(UR + 1, nd);
    const double DL = UL[0] * (SL - uL);
    const double DR = UR[0] * (SR - uR);
    const double num = (wr.p - wl.p) + __builtin_fma(mL, SL - uL, -(mR * (SR - uR)));
    const double den = DL - DR;
    const double Ss = num / den;
    const bool left = (Ss >= 0.0);
    const double SK = left ? SL : SR;
    const double DK = left ? DL : DR;
    const double uK = left ? uL : uR;
    const double pK = left ? wl.p : wr.p;
    const double irK = left ? wl.ir : wr.ir;
    const double f = DK / (SK - Ss);
    double Us[NF], UK[NF], FK[NF];
#pragma unroll
    for (int q = 0; q < NF; ++q) {
        UK[q] = left ? UL[q] : UR[q];
        FK[q] = left ? FL[q] : FR[q];
    }
    Us[0] = f;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        const double vk = left ? wl.u[k] : wr.u[k];
        Us[1 + k] = (k == nd) ? (f * Ss) : (f * vk);
    }
    Us[DIM + 1] = f * __builtin_fma(UK[DIM + 1], irK, (Ss - uK) * (Ss + (pK / DK)));
#pragma unroll
    for (int q = 0; q < NF; ++q) {
        const double star = __builtin_fma(SK, Us[q] - UK[q], FK[q]);
        Fh[q] = takeL ? FL[q] : (takeR ? FR[q] : star);
    }
}

// ---------------------------------------------------------------- shallow water

// Shallow water (h, hu_1..hu_DIM): velocity hu_k (1/h), celerity sqrt(g h).
template <int DIM>
struct SwePrim {
    double ih;
    double u[DIM];
    double c;
};

template <int DIM>
__device__ __forceinline__ SwePrim<DIM> swe_prim(const double* U, const Phys& ph)
{
    SwePrim<DIM> w;
    w.ih = 1.0 / U[0];
#pragma unroll
    for (int k = 0; k < DIM; ++k) w.u[k] = U[1 + k] * w.ih;
    w.c = sqrt(ph.grav * U[0]);
    return w;
}

// Physical flux along nd: (hu_nd, hu_k u_nd + [k == nd] g h^2 / 2).
template <int DIM>
__device__ __forceinline__ void swe_flux(const double* U, const SwePrim<DIM>& w, int nd, double* F,
                                         const Phys& ph)
{
    const double un = pick<DIM>(w.u, nd);
    const double hp = 0.5 * (ph.grav * (U[0] * U[0]));
    F[0] = pick<DIM>(U + 1, nd);
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        const double a = U[1 + k] * un;
        F[1 + k] = (k == nd) ? (a + hp) : a;
    }
}

// Numerical flux of the shallow-water equations: Rusanov, HLL (Davis speeds u -+ c), or Roe
// (velocity averaged with sqrt(h) weights, celerity sqrt(g (h_L + h_R) / 2); gravity waves
// u -+ c with Harten's fix over half the jump of the one-sided speeds, shear waves at u;
// fields in the order u - c, shear (axes ascending), u + c).
template <int DIM, int FLUX>
__device__ __forceinline__ void swe_numflux(const double* UL, const double* UR, int nd, double* Fh,
                                            const Phys& ph)
{
    constexpr int NF = DIM + 1;
    const SwePrim<DIM> wl = swe_prim<DIM>(UL, ph);
    const SwePrim<DIM> wr = swe_prim<DIM>(UR, ph);
    double FL[NF], FR[NF];
    swe_flux<DIM>(UL, wl, nd, FL, ph);
    swe_flux<DIM>(UR, wr, nd, FR, ph);
    const double uL = pick<DIM>(wl.u, nd), uR = pick<DIM>(wr.u, nd);
    if (FLUX == FLUX_RUSANOV) {
        const double s = vmax(fabs(uL) + wl.c, fabs(uR) + wr.c);
#pragma unroll
        for (int q = 0; q < NF; ++q) Fh[q] = 0.5 * ((FL[q] + FR[q]) - (s * (UR[q] - UL[q])));
        return;
    }
    if (FLUX == FLUX_ROE) {
        const double sqL = sqrt(UL[0]);
        const double sqR = sqrt(UR[0]);
        const double wsum = sqL + sqR;
        double ua[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) ua[k] = ((sqL * wl.u[k]) + (sqR * wr.u[k])) / wsum;
        const double ca = sqrt(ph.grav * (0.5 * (UL[0] + UR[0])));
        const double una = pick<DIM>(ua, nd);
        const double jh = UR[0] - UL[0];
        const double jq = (pick<DIM>(UR + 1, nd) - pick<DIM>(UL + 1, nd)) - (una * jh);
        const double s1 = 0.5 * (jh - (jq / ca));
        const double s2 = 0.5 * (jh + (jq / ca));
        const double fan1 = 0.5 * vmax(0.0, (uR - wr.c) - (uL - wl.c));
        const double fan2 = 0.5 * vmax(0.0, (uR + wr.c) - (uL + wl.c));
        const double g1 = harten_fix(una - ca, fan1) * s1;
        const double g2 = harten_fix(una + ca, fan2) * s2;
        double diss[NF];
        diss[0] = g1 + g2;
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            const bool n = (k == nd);
            double t = g1 * (n ? (una - ca) : ua[k]);
            t = n ? t : (t + (fabs(una) * ((UR[1 + k] - UL[1 + k]) - (ua[k] * jh))));
            diss[1 + k] = t + (g2 * (n ? (una + ca) : ua[k]));
        }
#pragma unroll
        for (int q = 0; q < NF; ++q) Fh[q] = 0.5 * ((FL[q] + FR[q]) - diss[q]);
        return;
    }
    const double SL = vmin(uL - wl.c, uR - wr.c);
    const double SR = vmax(uL + wl.c, uR + wr.c);
    const bool takeL = (SL >= 0.0);
    const bool takeR = (SR <= 0.0);
    const double den = SR - SL;
    const double slsr = SL * SR;
#pragma unroll
    for (int q = 0; q < NF; ++q) {
        const double mid = (((SR * FL[q]) - (SL * FR[q])) + (slsr * (UR[q] - UL[q]))) / den;
        Fh[q] = takeL ? FL[q] : (takeR ? FR[q] : mid);
    }
}

// ---------------------------------------------------------------- ideal MHD

// Ideal MHD (rho, m_x, m_y, m_z, E, B_x, B_y, B_z) in every dimension, magnetic pressure
// |B|^2 / 2: velocity m_k (1/rho), magnetic pressure pb, gas pressure
// (gamma - 1)((E - rho |u|^2 / 2) - pb).
struct MhdPrim {
    double ir;
    double u[3];
    double pb;
    double p;
};

__device__ __forceinline__ MhdPrim mhd_prim(const double* U, const Phys& ph)
{
    MhdPrim w;
    w.ir = 1.0 / U[0];
#pragma unroll
    for (int k = 0; k < 3; ++k) w.u[k] = U[1 + k] * w.ir;
    const double ke = 0.5 * (((U[1] * w.u[0]) + (U[2] * w.u[1])) + (U[3] * w.u[2]));
    w.pb = 0.5 * (((U[5] * U[5]) + (U[6] * U[6])) + (U[7] * U[7]));
    w.p = ph.gm1 * ((U[4] - ke) - w.pb);
    return w;
}

// Fast magnetosonic speed along axis nd: c_f^2 = (a^2 + b^2 + sqrt((a^2 + b^2)^2 -
// 4 a^2 b_n^2)) / 2, a^2 = gamma p / rho, b^2 = |B|^2 / rho, b_n^2 = B_n^2 / rho.
__device__ __forceinline__ double mhd_fast(const double* U, const MhdPrim& w, int nd, const Phys& ph)
{
    const double a2 = (ph.gamma * w.p) * w.ir;
    const double b2 = (2.0 * w.pb) * w.ir;
    const double bn = (nd == 0) ? U[5] : ((nd == 1) ? U[6] : U[7]);
    const double bn2 = (bn * bn) * w.ir;
    const double s = a2 + b2;
    const double disc = vmax(0.0, (s * s) - ((4.0 * a2) * bn2));
    return sqrt(0.5 * (s + sqrt(disc)));
}

// Ideal MHD flux along nd: m_n; m_k u_n - B_n B_k (+ p + pb on k = nd);
// (E + p + pb) u_n - B_n (u . B); u_n B_k - B_n u_k.
__device__ __forceinline__ void mhd_flux(const double* U, const MhdPrim& w, int nd, double* F)
{
    const double un = (nd == 0) ? w.u[0] : ((nd == 1) ? w.u[1] : w.u[2]);
    const double bn = (nd == 0) ? U[5] : ((nd == 1) ? U[6] : U[7]);
    const double pt = w.p + w.pb;
    const double ub = ((w.u[0] * U[5]) + (w.u[1] * U[6])) + (w.u[2] * U[7]);
    F[0] = (nd == 0) ? U[1] : ((nd == 1) ? U[2] : U[3]);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double f = (U[1 + k] * un) - (bn * U[5 + k]);
        F[1 + k] = (k == nd) ? (f + pt) : f;
        F[5 + k] = (un * U[5 + k]) - (bn * w.u[k]);
    }
    F[4] = ((U[4] + pt) * un) - (bn * ub);
}

// Numerical flux of ideal MHD: Rusanov or HLL on the fast magnetosonic speeds (Davis).
template <int FLUX>
__device__ __forceinline__ void mhd_numflux(const double* UL, const double* UR, int nd, double* Fh,
                                            const Phys& ph)
{
    static_assert(FLUX == FLUX_RUSANOV || FLUX == FLUX_HLL, "ideal MHD: Rusanov or HLL");
    const MhdPrim wl = mhd_prim(UL, ph);
    const MhdPrim wr = mhd_prim(UR, ph);
    double FL[8], FR[8];
    mhd_flux(UL, wl, nd, FL);
    mhd_flux(UR, wr, nd, FR);
    const double uL = (nd == 0) ? wl.u[0] : ((nd == 1) ? wl.u[1] : wl.u[2]);
    const double uR = (nd == 0) ? wr.u[0] : ((nd == 1) ? wr.u[1] : wr.u[2]);
    const double cL = mhd_fast(UL, wl, nd, ph), cR = mhd_fast(UR, wr, nd, ph);
    if (FLUX == FLUX_RUSANOV) {
        const double s = vmax(fabs(uL) + cL, fabs(uR) + cR);
#pragma unroll
        for (int q = 0; q < 8; ++q) Fh[q] = 0.5 * ((FL[q] + FR[q]) - (s * (UR[q] - UL[q])));
        return;
    }
    const double SL = vmin(uL - cL, uR - cR);
    const double SR = vmax(uL + cL, uR + cR);
    const bool takeL = (SL >= 0.0);
    const bool takeR = (SR <= 0.0);
    const double den = SR - SL;
    const double slsr = SL * SR;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const double mid = (((SR * FL[q]) - (SL * FR[q])) + (slsr * (UR[q] - UL[q]))) / den;
        Fh[q] = takeL ? FL[q] : (takeR ? FR[q] : mid);
    }
}

// ---------------------------------------------------------------- scalar equations

template <int DIM, int EQ, int FLUX>
__device__ __forceinline__ double scalar_numflux(double uL, double uR, int nd, const Phys& ph)
{
    double FL, FR, s, SL, SR;
    if (EQ == EQ_BURGERS) {
        FL = 0.5 * (uL * uL);
        FR = 0.5 * (uR * uR);
        s = vmax(fabs(uL), fabs(uR));
        SL = vmin(uL, uR);
        SR = vmax(uL, uR);
    } else {
        const double a = pick<DIM>(ph.vel, nd);
        FL = a * uL;
        FR = a * uR;
        s = fabs(a);
        SL = a;
        SR = a;
    }
    if (FLUX == FLUX_RUSANOV) return 0.5 * ((FL + FR) - (s * (uR - uL)));
    if (FLUX == FLUX_ROE) {
        // Roe speed: the mean for Burgers, with the fix over a rarefaction fan; the velocity
        // for advection (plain upwinding)
        const double a = (EQ == EQ_BURGERS) ? (0.5 * (uL + uR)) : SL;
        const double fan = (EQ == EQ_BURGERS) ? (0.5 * vmax(0.0, uR - uL)) : 0.0;
        return 0.5 * ((FL + FR) - (harten_fix(a, fan) * (uR - uL)));
    }
    if (FLUX == FLUX_EC || FLUX == FLUX_EC4)                                   // Burgers
        return (((uL * uL) + (uL * uR)) + (uR * uR)) / 6.0;
    if (FLUX == FLUX_GODUNOV) {
        // exact Riemann solution at x/t = 0: for Burgers a shock (uL > uR) goes the way of its
        // speed (uL + uR)/2, a fan containing 0 gives f(0) = 0; advection upwinds
        if (EQ == EQ_BURGERS) {
            if (uL > uR) return ((0.5 * (uL + uR)) >= 0.0) ? FL : FR;
            return (uL >= 0.0) ? FL : ((uR <= 0.0) ? FR : 0.0);
        }
        return (SL >= 0.0) ? FL : FR;
    }
    const double mid = (((SR * FL) - (SL * FR)) + ((SL * SR) * (uR - uL))) / (SR - SL);
    return (SL >= 0.0) ? FL : ((SR <= 0.0) ? FR : mid);
}

template <int DIM, int EQ, int FLUX>
__device__ __forceinline__ void numflux(const double* UL, const double* UR, int nd, double* Fh,
                                        const Phys& ph)
{
    if constexpr (EQ == EQ_EULER) {
        euler_numflux<DIM, FLUX>(UL, UR, nd, Fh, ph);
    } else if constexpr (EQ == EQ_SWE) {
        swe_numflux<DIM, FLUX>(UL, UR, nd, Fh, ph);
    } else if constexpr (EQ == EQ_MHD) {
        mhd_numflux<FLUX>(UL, UR, nd, Fh, ph);
    } else {
        Fh[0] = scalar_numflux<DIM, EQ, FLUX>(UL[0], UR[0], nd, ph);
    }
}

// Fourth-order entropy-conservative flux (LeFloch, Mercier and Rohde) at the face between
// cells B and C of the cell values A, B, C, D (i-1..i+2): the combination
// (4/3) F~(B, C) - (1/6) (F~(B, D) + F~(A, C)) of the two-point entropy-conservative flux F~.
template <int DIM, int EQ>
__device__ __forceinline__ void ec4_face(const double* A, const double* B, const double* C,
                                         const double* D, int nd, double* F, const Phys& ph)
{
    constexpr int NF = NumFields<DIM, EQ>::value;
    double F1[NF], F2[NF], F3[NF];
    if constexpr (EQ == EQ_EULER) {
        // the primitives and beta of each of the four cells once, for the three pairs
        const EulerPrim<DIM> wa = euler_prim<DIM>(A, ph), wb = euler_prim<DIM>(B, ph);
        const EulerPrim<DIM> wc = euler_prim<DIM>(C, ph), wd = euler_prim<DIM>(D, ph);
        const double ba = ec_beta<DIM>(A, wa), bb = ec_beta<DIM>(B, wb);
        const double bc = ec_beta<DIM>(C, wc), bd = ec_beta<DIM>(D, wd);
        ec_euler_flux<DIM>(B, C, wb, wc, bb, bc, nd, F1, ph);
        ec_euler_flux<DIM>(B, D, wb, wd, bb, bd, nd, F2, ph);
        ec_euler_flux<DIM>(A, C, wa, wc, ba, bc, nd, F3, ph);
    } else {
        numflux<DIM, EQ, FLUX_EC>(B, C, nd, F1, ph);
        numflux<DIM, EQ, FLUX_EC>(B, D, nd, F2, ph);
        numflux<DIM, EQ, FLUX_EC>(A, C, nd, F3, ph);
    }
#pragma unroll
    for (int q = 0; q < NF; ++q) F[q] = ((4.0 / 3.0) * F1[q]) - ((1.0 / 6.0) * (F2[q] + F3[q]));
}

// ---------------------------------------------------------------- reconstruction

__device__ __forceinline__ double minmod(double a, double b)
{
    return (a > 0.0 && b > 0.0) ? vmin(a, b) : ((a < 0.0 && b < 0.0) ? vmax(a, b) : 0.0);
}

// Third-order WENO (Jiang--Shu indicators, eps = 1e-6, power 2): the value at the face
// between b and c from cells (a, b, c), candidates (b+c)/2 and (3b-a)/2 with linear weights
// 2/3 and 1/3, combined with a single division. The smoothness terms, the candidate (3b-a)/2
// and the numerator are fused multiply-adds (one rounding each).
__device__ __forceinline__ double weno3(double a, double b, double c)
{
    const double d0 = b - a;
    const double d1 = c - b;
    double t0 = __builtin_fma(d1, d1, 1e-6);
    t0 = t0 * t0;
    double t1 = __builtin_fma(d0, d0, 1e-6);
    t1 = t1 * t1;
    const double q0 = 0.5 * (b + c);
    const double q1 = __builtin_fma(1.5, b, -(0.5 * a));
    return __builtin_fma(2.0 * t1, q0, t0 * q1) / ((2.0 * t1) + t0);
}

// Left and right states at the face between cells i-1 and i from the stencil
// (a, b, c, d) = (U_{i-2}, U_{i-1}, U_i, U_{i+1}) of one conserved component.
template <int RECON>
__device__ __forceinline__ void reconstruct(double a, double b, double c, double d,
                                            double& uL, double& uR)
{
    if (RECON == REC_FIRST) {
        uL = b;
        uR = c;
    } else if (RECON == REC_MUSCL) {
        uL = b + (0.5 * minmod(b - a, c - b));
        uR = c - (0.5 * minmod(c - b, d - c));
    } else if (RECON == REC_ENO2) {
        // the one-sided difference of smaller magnitude (the left one on a tie)
        const double lb = b - a, rb = c - b, rc = d - c;
        uL = b + (0.5 * ((fabs(lb) <= fabs(rb)) ? lb : rb));
        uR = c - (0.5 * ((fabs(rb) <= fabs(rc)) ? rb : rc));
    } else {
        // uL = weno3(a, b, c), uR = weno3(d, c, b). Both use the indicator of (b, c) and the
        // candidate (b + c)/2: (b - c)^2 equals (c - b)^2 and b + c equals c + b bit for bit,
        // so each is computed once.
        const double dbc = c - b;
        double tbc = __builtin_fma(dbc, dbc, 1e-6);
        tbc = tbc * tbc;
        const double q0 = 0.5 * (b + c);
        const double dab = b - a;
        double tab = __builtin_fma(dab, dab, 1e-6);
        tab = tab * tab;
        const double q1L = __builtin_fma(1.5, b, -(0.5 * a));
        uL = __builtin_fma(2.0 * tab, q0, tbc * q1L) / ((2.0 * tab) + tbc);
        const double ddc = c - d;
        double tdc = __builtin_fma(ddc, ddc, 1e-6);
        tdc = tdc * tdc;
        const double q1R = __builtin_fma(1.5, c, -(0.5 * d));
        uR = __builtin_fma(2.0 * tdc, q0, tbc * q1R) / ((2.0 * tdc) + tbc);
    }
}

// ---------------------------------------------------------------- wave speed

// max over axes of (|u_k| + c) / dx_k (Euler), |u| / dx_k (Burgers), |a_k| / dx_k
// (advection) for one cell; *bad set when the state is non-physical.
template <int DIM, int EQ>
__device__ __forceinline__ double cell_speed(const double* U, const Phys& ph, bool& bad)
{
    constexpr int NF = NumFields<DIM, EQ>::value;
    bool b = false;
#pragma unroll
    for (int q = 0; q < NF; ++q) b = b || !isfinite(U[q]);
    double m = 0.0;
    if constexpr (EQ == EQ_EULER) {
        const EulerPrim<DIM> w = euler_prim<DIM>(U, ph);
        b = b || !(U[0] > 0.0) || !(w.p > 0.0);
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            const double a = (fabs(w.u[k]) + w.c) * ph.inv_dx[k];
            m = (k == 0) ? a : vmax(m, a);
        }
    } else if constexpr (EQ == EQ_MHD) {
        const MhdPrim w = mhd_prim(U, ph);
        b = b || !(U[0] > 0.0) || !(w.p > 0.0);
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            const double a = (fabs(w.u[k]) + mhd_fast(U, w, k, ph)) * ph.inv_dx[k];
            m = (k == 0) ? a : vmax(m, a);
        }
    } else if constexpr (EQ == EQ_SWE) {
        const SwePrim<DIM> w = swe_prim<DIM>(U, ph);
        b = b || !(U[0] > 0.0);
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            const double a = (fabs(w.u[k]) + w.c) * ph.inv_dx[k];
            m = (k == 0) ? a : vmax(m, a);
        }
    } else {
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            const double s = (EQ == EQ_BURGERS) ? fabs(U[0]) : fabs(ph.vel[k]);
            const double a = s * ph.inv_dx[k];
            m = (k == 0) ? a : vmax(m, a);
        }
    }
    bad = b;
    return m;
}

}  // namespace fvk
