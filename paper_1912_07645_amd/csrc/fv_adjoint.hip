// fv_adjoint.hip -- discrete adjoint of the finite-volume scheme: the transpose of the
// linearised Runge--Kutta stage (reconstruction -> Rusanov flux -> divergence) for the
// Euler equations, the kinetic-energy quantity of interest, and the contraction of the
// initial-state adjoint with the derivative of line-wise initial data.
//
// The reverse stage is in gather form. With L_i = -sum_k (F_{i+1/2} - F_{i-1/2}) / dx_k,
// sum_i lam_i . L_i = sum_faces F_f . w_f, w_f = (lam_right - lam_left) / dx. Every face
// therefore contributes (dF_f / dU_c)^T w_f to the four cells c of its stencil, through
// g_L = (dF/dU_L)^T w and g_R = (dF/dU_R)^T w and the reconstruction's partial derivatives.
// The faces of a tile store (g_L, g_R, minmod branch codes) in LDS, one axis at a time; each
// cell then adds that axis's four faces in a fixed order, with no atomics, so results are
// reproducible.
// Branches follow the forward pass: the larger Rusanov speed (ties to the right state), the
// minmod argument selected (ties as the forward comparison), sign(0) = 0 for |u|.
#include "fv_adjoint.h"
#include "fv_stage.h"

namespace fvk {

// (A^T w) for the Euler flux along nd at state U: A = dF/dU.
template <int DIM>
__device__ __forceinline__ void euler_flux_jt(const double* U, const EulerPrim<DIM>& pr, int nd,
                                              const double* w, const Phys& ph, double* out)
{
    constexpr int NF = DIM + 2;
    const double un = pick<DIM>(pr.u, nd);
    const double H = (U[NF - 1] + pr.p) * pr.ir;           // (E + p) / rho
    double usq = 0.0, S = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        usq = usq + pr.u[k] * pr.u[k];
        S = S + w[1 + k] * pr.u[k];
    }
    const double p_rho = ph.gm1 * (0.5 * usq);
    const double p_E = ph.gm1;
    const double wn = pick<DIM>(w + 1, nd);
    const double wE = w[NF - 1];
    const double Wp = wn + wE * un;
    out[0] = -un * (S + wE * H) + Wp * p_rho;
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
        const double pm = -ph.gm1 * pr.u[j];
        double v = w[1 + j] * un + Wp * pm;
        if (j == nd) v = v + (w[0] + S + wE * H);
        out[1 + j] = v;
    }
    out[NF - 1] = wE * un + Wp * p_E;
}

// Gradient of |u_n| + c with respect to U.
template <int DIM>
__device__ __forceinline__ void speed_grad(const double* U, const EulerPrim<DIM>& pr, int nd,
                                           const Phys& ph, double* g)
{
    constexpr int NF = DIM + 2;
    const double un = pick<DIM>(pr.u, nd);
    const double sg = (un > 0.0) ? 1.0 : ((un < 0.0) ? -1.0 : 0.0);
    double usq = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) usq = usq + pr.u[k] * pr.u[k];
    const double a = ph.gamma / (2.0 * pr.c * U[0]);       // dc/dp
    const double p_rho = ph.gm1 * (0.5 * usq);
    g[0] = sg * (-un * pr.ir) + (a * p_rho - pr.c / (2.0 * U[0]));
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        double v = a * (-ph.gm1 * pr.u[k]);
        if (k == nd) v = v + sg * pr.ir;
        g[1 + k] = v;
    }
    g[NF - 1] = a * ph.gm1;
}

// minmod branch: 0 -> 0, 1 -> first argument, 2 -> second (as the forward comparisons).
__device__ __forceinline__ int minmod_code(double a, double b)
{
    if (a > 0.0 && b > 0.0) return (a < b) ? 1 : 2;
    if (a < 0.0 && b < 0.0) return (a > b) ? 1 : 2;
    return 0;
}

// SplitMix64's finaliser (Steele, Lea and Flood 2014): hashes the branch-signature terms.
__device__ __forceinline__ unsigned long long sig_mix(unsigned long long z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <int DIM, int RECON, int BX, int BY, int NT>
struct AdjTile {
    static constexpr int NF = DIM + 2;
    static constexpr int R = (RECON == REC_MUSCL) ? 1 : 0;  // extra faces per side
    static constexpr int HU = (RECON == REC_MUSCL) ? 3 : 1;  // halo of U
    static constexpr int HL = (RECON == REC_MUSCL) ? 2 : 1;  // halo of lambda
    static constexpr int UX = BX + 2 * HU, UY = (DIM >= 2) ? BY + 2 * HU : 1;
    static constexpr int LX = BX + 2 * HL, LY = (DIM >= 2) ? BY + 2 * HL : 1;
    // x faces: right-cell index k in [x0 - R, x0 + BX + R], all rows of the tile
    static constexpr int EXN = BX + 1 + 2 * R;
    static constexpr int NFX = EXN * BY;
    static constexpr int EYN = (DIM >= 2) ? BY + 1 + 2 * R : 0;
    static constexpr int NFY = (DIM >= 2) ? BX * EYN : 0;
    static constexpr int NFACES = NFX + NFY;
    static constexpr int CELLS = BX * BY;
    static constexpr int CPT = (CELLS + NT - 1) / NT;
};

template <int DIM, int RECON, int BX, int BY, int NT>
__global__ void __launch_bounds__(NT)
adjoint_stage_kernel(const AdjArgs a)
{
    using T = AdjTile<DIM, RECON, BX, BY, NT>;
    constexpr int NF = T::NF, R = T::R, HU = T::HU, HL = T::HL;
    constexpr int UX = T::UX, UY = T::UY, LX = T::LX, LY = T::LY;
    constexpr int NFX = T::NFX, NFACES = T::NFACES, EXN = T::EXN, EYN = T::EYN;
    constexpr int UC = UX * UY, LC = LX * LY;
    constexpr int NFY = T::NFY;
    constexpr int MAXF = NFX > NFY ? NFX : NFY;   // faces of one axis
    __shared__ double su[NF * UC];
    __shared__ double sl[NF * LC];
    __shared__ double sg[2 * NF * MAXF];   // g_L, g_R per face of the axis in hand
    __shared__ int scode[MAXF];            // minmod codes, 2 bits per component and side
    __shared__ unsigned long long ssig;    // the workgroup's branch-signature sum

    const int64_t blk = xcd_remap(blockIdx.x, a.nblocks);
    const int32_t sample = (int32_t)(blk / a.ntiles);
    const int32_t tile = (int32_t)(blk % a.ntiles);
    const int32_t tx = tile % a.tiles[0];
    const int32_t ty = tile / a.tiles[0];
    const int32_t x0 = tx * BX, y0 = ty * BY;
    const int32_t nx = a.n[0], ny = a.n[1];
    const int64_t sbase = (int64_t)sample * NF * a.cells;
    const double* U = a.U + sbase;
    const double* lam = a.lam + sbase;

    // the haloed tiles of U and lambda into LDS, every load issued before the first store
    {
        constexpr int UPT = (UC + NT - 1) / NT, LPT = (LC + NT - 1) / NT;
        double vu[UPT][NF], vl[LPT][NF];
#pragma unroll
        for (int k = 0; k < UPT; ++k) {
            const int e = threadIdx.x + k * NT;
            if ((k + 1) * NT <= UC || e < UC) {
                const int px = e % UX, py = e / UX;
                const int32_t gx = wrap_index(x0 + px - HU, nx, a.bc[0]);
                const int32_t gy = (DIM >= 2) ? wrap_index(y0 + py - HU, ny, a.bc[1]) : 0;
                const int32_t gi = gy * nx + gx;   // cells < 2^31
#pragma unroll
                for (int q = 0; q < NF; ++q) vu[k][q] = U[q * a.cells + gi];
            }
        }
#pragma unroll
        for (int k = 0; k < LPT; ++k) {
            const int e = threadIdx.x + k * NT;
            if ((k + 1) * NT <= LC || e < LC) {
                const int px = e % LX, py = e / LX;
                const int32_t gx = wrap_index(x0 + px - HL, nx, a.bc[0]);
                const int32_t gy = (DIM >= 2) ? wrap_index(y0 + py - HL, ny, a.bc[1]) : 0;
                const int32_t gi = gy * nx + gx;
#pragma unroll
                for (int q = 0; q < NF; ++q) vl[k][q] = lam[q * a.cells + gi];
            }
        }
#pragma unroll
        for (int k = 0; k < UPT; ++k) {
            const int e = threadIdx.x + k * NT;
            if ((k + 1) * NT <= UC || e < UC) {
#pragma unroll
                for (int q = 0; q < NF; ++q) su[q * UC + e] = vu[k][q];
            }
        }
#pragma unroll
        for (int k = 0; k < LPT; ++k) {
            const int e = threadIdx.x + k * NT;
            if ((k + 1) * NT <= LC || e < LC) {
#pragma unroll
                for (int q = 0; q < NF; ++q) sl[q * LC + e] = vl[k][q];
            }
        }
    }
    __syncthreads();

    // one axis at a time: its faces' (g_L, g_R, codes) into LDS, then every cell gathers the
    // axis's four (MUSCL) or two faces; axis 0 is added before axis 1, as in eq. 2.1
    double jt[T::CPT][NF];
#pragma unroll
    for (int k = 0; k < T::CPT; ++k)
#pragma unroll
        for (int q = 0; q < NF; ++q) jt[k][q] = 0.0;
    unsigned long long hsig = 0ull;   // this thread's signature terms (faces it owns)
#pragma unroll
    for (int nd = 0; nd < DIM; ++nd) {
        const int nfaces = (nd == 0) ? NFX : NFY;
        for (int f = threadIdx.x; f < nfaces; f += NT) {
            int fx, fy;   // face between (right cell) and (right cell - e_nd), tile-local
            if (nd == 0) {
                fx = f % EXN - R;          // right-cell x offset from x0, in [-R, BX + R]
                fy = f / EXN;
            } else {
                fx = f % BX;
                fy = f / BX - R;
            }
            const int cu = ((DIM >= 2 ? fy + HU : 0)) * UX + (fx + HU);
            const int su_stride = (nd == 0) ? 1 : UX;
            const int cl = ((DIM >= 2 ? fy + HL : 0)) * LX + (fx + HL);
            const int sl_stride = (nd == 0) ? 1 : LX;
            double UL[NF], UR[NF], w[NF];
            int codes = 0;
            const double inv = (nd == 0) ? a.ph.inv_dx[0] : a.ph.inv_dx[1];
#pragma unroll
            for (int q = 0; q < NF; ++q) {
                const double* sp = su + q * UC + cu;
                const double ua = sp[-su_stride], ub = sp[0];
                if (RECON == REC_MUSCL) {
                    const double uam = sp[-2 * su_stride], ubp = sp[su_stride];
                    const int cL = minmod_code(ua - uam, ub - ua);
                    const int cR = minmod_code(ub - ua, ubp - ub);
                    codes |= (cL | (cR << 2)) << (4 * q);
                    UL[q] = ua + (0.5 * minmod(ua - uam, ub - ua));
                    UR[q] = ub - (0.5 * minmod(ub - ua, ubp - ub));
                } else {
                    UL[q] = ua;
                    UR[q] = ub;
                }
                const double* l = sl + q * LC + cl;
                w[q] = inv * (l[0] - l[-sl_stride]);
            }
            const EulerPrim<DIM> pl = euler_prim<DIM>(UL, a.ph);
            const EulerPrim<DIM> pr = euler_prim<DIM>(UR, a.ph);
            const double sL = fabs(pick<DIM>(pl.u, nd)) + pl.c;
            const double sR = fabs(pick<DIM>(pr.u, nd)) + pr.c;
            const bool selL = sL > sR;
            const double s = selL ? sL : sR;
            double jl[NF], jr[NF], gs[NF];
            euler_flux_jt<DIM>(UL, pl, nd, w, a.ph, jl);
            euler_flux_jt<DIM>(UR, pr, nd, w, a.ph, jr);
            if (selL) speed_grad<DIM>(UL, pl, nd, a.ph, gs);
            else speed_grad<DIM>(UR, pr, nd, a.ph, gs);
            double wd = 0.0;
#pragma unroll
            for (int q = 0; q < NF; ++q) wd = wd + w[q] * (UR[q] - UL[q]);
#pragma unroll
            for (int q = 0; q < NF; ++q) {
                const double ds = 0.5 * wd * gs[q];
                const double gL = 0.5 * (jl[q] + s * w[q]) - (selL ? ds : 0.0);
                const double gR = 0.5 * (jr[q] - s * w[q]) - (selL ? 0.0 : ds);
                sg[(2 * q) * MAXF + f] = gL;
                sg[(2 * q + 1) * MAXF + f] = gR;
            }
            scode[f] = codes;
            if (a.sig) {
                // each face once: by the tile of its right cell, inside the grid
                const int32_t gx = x0 + fx, gy = (DIM >= 2) ? y0 + fy : 0;
                const bool own = (nd == 0) ? (fx >= 0 && fx < BX) : (fy >= 0 && fy < BY);
                if (own && gx < nx && gy < ny) {
                    const double un = selL ? pick<DIM>(pl.u, nd) : pick<DIM>(pr.u, nd);
                    const unsigned long long sgn = (un > 0.0) ? 2ull : ((un < 0.0) ? 0ull : 1ull);
                    const unsigned long long code = (unsigned long long)(unsigned)codes |
                                                    ((selL ? 1ull : 0ull) << 32) | (sgn << 33);
                    const unsigned long long key = ((unsigned long long)(gy * nx + gx) << 2) | nd;
                    hsig += sig_mix(a.salt ^ sig_mix(key * 0x9E3779B97F4A7C15ull + code));
                }
            }
        }
        __syncthreads();

#pragma unroll
        for (int k = 0; k < T::CPT; ++k) {
            const int c = threadIdx.x + k * NT;
            if (c >= T::CELLS) break;
            const int cx = c % BX, cy = c / BX;
            // face index (within this axis) with right cell at tile offset o + shift along nd
            auto face = [&](int shift) -> int {
                if (nd == 0) return cy * EXN + (cx + shift + R);
                return (cy + shift + R) * BX + cx;
            };
#pragma unroll
            for (int q = 0; q < NF; ++q) {
                double v = jt[k][q];
                if (RECON == REC_MUSCL) {
                    {   // face c - 3/2 (right cell c - 1): this cell is b + 1
                        const int f = face(-1);
                        const int cR = (scode[f] >> (4 * q + 2)) & 3;
                        v = v + sg[(2 * q + 1) * MAXF + f] * ((cR == 2) ? -0.5 : 0.0);
                    }
                    {   // face c - 1/2 (right cell c): this cell is b
                        const int f = face(0);
                        const int cL = (scode[f] >> (4 * q)) & 3;
                        const int cR = (scode[f] >> (4 * q + 2)) & 3;
                        v = v + sg[(2 * q) * MAXF + f] * ((cL == 2) ? 0.5 : 0.0);
                        v = v + sg[(2 * q + 1) * MAXF + f] * ((cR == 1) ? 0.5 : ((cR == 2) ? 1.5 : 1.0));
                    }
                    {   // face c + 1/2 (right cell c + 1): this cell is a
                        const int f = face(1);
                        const int cL = (scode[f] >> (4 * q)) & 3;
                        const int cR = (scode[f] >> (4 * q + 2)) & 3;
                        v = v + sg[(2 * q) * MAXF + f] * ((cL == 1) ? 1.5 : ((cL == 2) ? 0.5 : 1.0));
                        v = v + sg[(2 * q + 1) * MAXF + f] * ((cR == 1) ? 0.5 : 0.0);
                    }
                    {   // face c + 3/2 (right cell c + 2): this cell is a - 1
                        const int f = face(2);
                        const int cL = (scode[f] >> (4 * q)) & 3;
                        v = v + sg[(2 * q) * MAXF + f] * ((cL == 1) ? -0.5 : 0.0);
                    }
                } else {
                    v = v + sg[(2 * q + 1) * MAXF + face(0)];   // face c - 1/2: g_R
                    v = v + sg[(2 * q) * MAXF + face(1)];       // face c + 1/2: g_L
                }
                jt[k][q] = v;
            }
        }
        if (nd + 1 < DIM) __syncthreads();   // the next axis overwrites sg
    }
    if (a.sig) {   // uniform over the launch
        if (threadIdx.x == 0) ssig = 0ull;
        __syncthreads();
        atomicAdd(&ssig, hsig);
        __syncthreads();
        if (threadIdx.x == 0) atomicAdd(a.sig + sample, ssig);
    }

    // the reverse stage combination
    double* prev = a.prev + sbase;
    double* acc = a.acc + sbase;
#pragma unroll
    for (int k = 0; k < T::CPT; ++k) {
        const int c = threadIdx.x + k * NT;
        if (c >= T::CELLS) break;
        const int cx = c % BX, cy = c / BX;
        const int32_t gx = x0 + cx, gy = y0 + cy;
        if (gx >= nx || gy >= ny) continue;
        const int32_t gi = gy * nx + gx;
        const int cl = ((DIM >= 2 ? cy + HL : 0)) * LX + (cx + HL);
#pragma unroll
        for (int q = 0; q < NF; ++q) {
            const double lq = sl[q * LC + cl];
            const double contrib = a.beta * (lq + a.dt * jt[k][q]);
            const int64_t o = q * a.cells + gi;
            if (a.mode == 2) {
                prev[o] = acc[o] + contrib;
            } else {
                prev[o] = contrib;
                const double keep = (1.0 - a.beta) * lq;
                acc[o] = (a.mode == 0) ? keep : (acc[o] + keep);
            }
        }
    }
}

template <int DIM, int RECON, int BX, int BY, int NT>
void launch_adjoint(const AdjArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL((adjoint_stage_kernel<DIM, RECON, BX, BY, NT>), dim3((unsigned)a.nblocks),
                       dim3(NT), 0, s, a);
}

struct AdjEntry {
    int dim, recon;
    AdjKernel k;
};

static const AdjEntry kAdj[] = {
    {1, REC_FIRST, {&launch_adjoint<1, REC_FIRST, 255, 1, 256>, 255, 1, 1}},
    {1, REC_MUSCL, {&launch_adjoint<1, REC_MUSCL, 253, 1, 256>, 253, 1, 1}},
    {2, REC_FIRST, {&launch_adjoint<2, REC_FIRST, 16, 15, 256>, 16, 15, 1}},
    {2, REC_MUSCL, {&launch_adjoint<2, REC_MUSCL, 16, 13, 256>, 16, 13, 1}},
};

const AdjKernel* find_adjoint_kernel(int dim, int eq, int recon, int flux)
{
    if (eq != EQ_EULER || flux != FLUX_RUSANOV) return nullptr;
    for (const AdjEntry& e : kAdj)
        if (e.dim == dim && e.recon == recon) return &e.k;
    return nullptr;
}

// ------------------------------------------------------------------ quantity of interest

constexpr int kQoiCells = 4096;

int qoi_blocks(int64_t cells) { return (int)((cells + kQoiCells - 1) / kQoiCells); }

template <int DIM>
__global__ void __launch_bounds__(256)
qoi_ke_kernel(const double* __restrict__ state, int32_t nx, int32_t ny, int32_t nz, int32_t j0,
              int32_t j1, double volume, const double* __restrict__ seed, double* __restrict__ grad,
              double* __restrict__ partial, int32_t nblk)
{
    constexpr int NF = DIM + 2;
    __shared__ double red[256];
    const int64_t cells = (int64_t)nx * ny * nz;
    const int blk = blockIdx.x;
    const int32_t b = blockIdx.y;
    const double* U = state + (int64_t)b * NF * cells;
    const double g = seed ? seed[b] : 0.0;
    double acc = 0.0;
    const int64_t c0 = (int64_t)blk * kQoiCells;
    for (int64_t c = c0 + threadIdx.x; c < c0 + kQoiCells && c < cells; c += 256) {
        const int32_t j = (int32_t)((c / nx) % ny);
        const bool in = (j >= j0 && j < j1);
        double V[NF];
#pragma unroll
        for (int q = 0; q < NF; ++q) V[q] = U[q * cells + c];
        const double ir = 1.0 / V[0];
        double mm = V[1] * V[1];
#pragma unroll
        for (int k = 1; k < DIM; ++k) mm = mm + (V[1 + k] * V[1 + k]);
        if (in) acc = acc + (0.5 * (mm * ir));
        if (grad) {
            double* G = grad + (int64_t)b * NF * cells + c;
            const double s = in ? g * volume : 0.0;
            G[0] = s * (-0.5 * (mm * ir) * ir);
#pragma unroll
            for (int k = 0; k < DIM; ++k) G[(1 + k) * cells] = s * (V[1 + k] * ir);
            G[(NF - 1) * cells] = 0.0;
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[(int64_t)b * nblk + blk] = red[0];
}

__global__ void qoi_finish_kernel(const double* __restrict__ partial, int32_t nblk, int32_t batch,
                                  double volume, double* __restrict__ Q)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    double s = partial[(int64_t)b * nblk];
    for (int k = 1; k < nblk; ++k) s = s + partial[(int64_t)b * nblk + k];
    Q[b] = s * volume;
}

void launch_qoi_ke(const double* state, int32_t dim, const int32_t n[3], int32_t batch,
                   int32_t j0, int32_t j1, double volume, const double* seed, double* Q,
                   double* grad, double* partial, int32_t nblk, hipStream_t s)
{
    const dim3 grid((unsigned)nblk, (unsigned)batch);
    if (dim == 1)
        hipLaunchKernelGGL(qoi_ke_kernel<1>, grid, dim3(256), 0, s, state, n[0], n[1], n[2], j0, j1,
                           volume, seed, grad, partial, nblk);
    else if (dim == 2)
        hipLaunchKernelGGL(qoi_ke_kernel<2>, grid, dim3(256), 0, s, state, n[0], n[1], n[2], j0, j1,
                           volume, seed, grad, partial, nblk);
    else
        hipLaunchKernelGGL(qoi_ke_kernel<3>, grid, dim3(256), 0, s, state, n[0], n[1], n[2], j0, j1,
                           volume, seed, grad, partial, nblk);
    if (Q)
        hipLaunchKernelGGL(qoi_finish_kernel, dim3((batch + 63) / 64), dim3(64), 0, s, partial, nblk,
                           batch, volume, Q);
}

// ------------------------------------------------------------------ line contraction

// One thread per (sample, line): sum over the line's cells (y order) and the fields.
__global__ void line_sum_kernel(const double* __restrict__ lam, const double* __restrict__ D,
                                int32_t nf, int32_t nx, int32_t ny, int32_t nz, int32_t batch,
                                double* __restrict__ sums)
{
    const int64_t lines = (int64_t)nx * nz;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= lines * batch) return;
    const int64_t b = t / lines, line = t % lines;
    const int64_t i = line % nx, k = line / nx;
    const int64_t cells = (int64_t)nx * ny * nz;
    const double* L = lam + b * nf * cells;
    const double* Dm = D + b * nf * cells;
    double s = 0.0;
    for (int32_t j = 0; j < ny; ++j) {
        const int64_t c = (k * ny + j) * nx + i;
        for (int q = 0; q < nf; ++q) s = s + L[q * cells + c] * Dm[q * cells + c];
    }
    sums[t] = s;
}

// One thread per (sample, parameter): sum over lines in order.
__global__ void line_theta_kernel(const double* __restrict__ sums, const double* __restrict__ E,
                                  int64_t lines, int32_t ntheta, int32_t batch,
                                  double* __restrict__ out)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntheta * batch) return;
    const int b = t / ntheta, k = t % ntheta;
    const double* S = sums + (int64_t)b * lines;
    const double* Eb = E + (int64_t)b * lines * ntheta;
    double acc = 0.0;
    for (int64_t l = 0; l < lines; ++l) acc = acc + S[l] * Eb[l * ntheta + k];
    out[t] = acc;
}

void launch_line_vjp(const double* lam, const double* D, const double* E, int32_t nf,
                     const int32_t n[3], int32_t batch, int32_t ntheta, double* line_sums,
                     double* out, hipStream_t s)
{
    const int64_t lines = (int64_t)n[0] * n[2];
    const int64_t t = lines * batch;
    hipLaunchKernelGGL(line_sum_kernel, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, s, lam, D,
                       nf, n[0], n[1], n[2], batch, line_sums);
    const int t2 = ntheta * batch;
    hipLaunchKernelGGL(line_theta_kernel, dim3((t2 + 63) / 64), dim3(64), 0, s, line_sums, E, lines,
                       ntheta, batch, out);
}

}  // namespace fvk
