// fv_stage_z.h -- the 3D Runge--Kutta stage kernel in its z-marching form.
//
// It computes exactly what the tiled stage kernel computes (same faces, same arithmetic, same
// order of the x, y, z divergence terms), but a workgroup owns a BX x BY block of columns and
// walks a segment of BZ planes along z, one plane at a time:
//   * each thread owns one column and keeps the 2G cells of that column that the next z face
//     reads in registers, so z faces need neither LDS nor re-reads of neighbouring planes; the
//     z flux on the lower face of a cell is the one the thread computed on the previous plane;
//   * only the current plane, with its x and y halo (no corners: faces read axis neighbours
//     only), is staged in LDS for the x and y faces; the plane's own cells come from the
//     column registers, so only the halo is loaded from memory for it;
//   * the next plane's halo and the next column cell are requested before the faces of the
//     current plane are computed, so their latency hides behind the arithmetic.
// A plane of a 16 x 15 block has 255 x faces, 256 y faces (two passes of 256 lanes) and one
// z face per column. Against a cube tile with a full halo this cuts the cells read per
// updated cell from (B + 2G)^3 / B^3 (4.6 for B = 6) to about 1.5, and the LDS per workgroup
// from 40 KB to 36 KB.
#pragma once

#include "fv_stage.h"

namespace fvk {

template <int EQ, int RECON, int BX, int BY, int NT>
struct ZTile {
    static constexpr int NF = NumFields<3, EQ>::value;
    static constexpr int G = Ghost<RECON>::value;
    static constexpr int PX = BX + 2 * G;
    static constexpr int PY = BY + 2 * G;
    static constexpr int PP = PX * PY;                    // plane cells with halo
    static constexpr int COLS = BX * BY;
    static constexpr int NH = 2 * G * (BX + BY);          // halo cells of a plane
    static constexpr int NFX = (BX + 1) * BY;
    static constexpr int NFY = BX * (BY + 1);
    static constexpr int NFXY = NFX + NFY;
    static constexpr int PXN = (NFX + 63) / 64 * 64;      // x faces padded to wavefronts
    static constexpr int PYN = (NFY + 63) / 64 * 64;
    static constexpr int TOTAL = PXN + PYN;
    static constexpr int FPT = (TOTAL + NT - 1) / NT;
    static_assert(NT % 64 == 0, "whole wavefronts");
    static_assert(COLS <= NT, "one column per thread");
    static_assert(NH <= NT, "one halo cell per thread");
};

// Position in the plane (with halo) of halo cell h: x halo (left, right), then y halo
// (bottom, top).
template <int G, int BX, int BY>
__device__ __forceinline__ void z_halo_pos(int h, int& px, int& py)
{
    if (h < 2 * G * BY) {
        const int side = h / (G * BY);
        const int r = h % (G * BY);
        py = G + r / G;
        px = (side == 0) ? (r % G) : (BX + G + r % G);
    } else {
        const int h2 = h - 2 * G * BY;
        const int side = h2 / (G * BX);
        const int r = h2 % (G * BX);
        px = G + r % BX;
        py = (side == 0) ? (r / BX) : (BY + G + r / BX);
    }
}

// One x (ND = 0) or y (ND = 1) face of the plane: reconstruction from LDS and flux.
template <int EQ, int RECON, int FLUX, int BX, int BY, int NT, int ND>
__device__ __forceinline__ void z_plane_face(const double* sp, const Phys& ph, int l, double* F)
{
    static_assert(FLUX != FLUX_EC4, "the z-marching kernel has no fourth-order EC path");
    using T = ZTile<EQ, RECON, BX, BY, NT>;
    constexpr int NF = T::NF, G = T::G, PX = T::PX, PP = T::PP;
    constexpr int EX = BX + (ND == 0);
    constexpr int STRIDE = (ND == 0) ? 1 : PX;
    const int fx = l % EX;
    const int fy = l / EX;
    const int c = (fy + G) * PX + (fx + G);
    double UL[NF], UR[NF];
#pragma unroll
    for (int q = 0; q < NF; ++q) {
        const double* s = sp + q * PP + c;
        if (RECON == REC_FIRST) {
            reconstruct<RECON>(0.0, s[-STRIDE], s[0], 0.0, UL[q], UR[q]);
        } else {
            reconstruct<RECON>(s[-2 * STRIDE], s[-STRIDE], s[0], s[STRIDE], UL[q], UR[q]);
        }
    }
    numflux<3, EQ, FLUX>(UL, UR, ND, F, ph);
}

// The z face above the window's middle: w[0..2G-1] are the column's cells k-G+1 .. k+G.
template <int EQ, int RECON, int FLUX, int NF, int G>
__device__ __forceinline__ void z_column_face(const double (&w)[2 * G][NF], const Phys& ph, double* F)
{
    double UL[NF], UR[NF];
#pragma unroll
    for (int q = 0; q < NF; ++q) {
        if (RECON == REC_FIRST) {
            reconstruct<RECON>(0.0, w[0][q], w[1][q], 0.0, UL[q], UR[q]);
        } else {
            reconstruct<RECON>(w[0][q], w[1][q], w[2][q], w[3][q], UL[q], UR[q]);
        }
    }
    numflux<3, EQ, FLUX>(UL, UR, 2, F, ph);
}

// WPE: the fewest wavefronts per SIMD to compile for. The column registers make this kernel
// need about 150 VGPRs (3 wavefronts per SIMD); at 4 some of them spill to scratch, and
// which costs less is measured. At 3, U^n is also requested a plane ahead.
template <int EQ, int RECON, int FLUX, int BX, int BY, int BZ, int NT, int WPE>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE, 8)))
stage_kernel_z(const StageArgs args)
{
    using T = ZTile<EQ, RECON, BX, BY, NT>;
    constexpr int NF = T::NF, G = T::G, PX = T::PX, PP = T::PP, COLS = T::COLS, NH = T::NH;
    constexpr int NFX = T::NFX, NFXY = T::NFXY;
    __shared__ double sp[NF * PP];     // current plane with its x and y halo
    __shared__ double sf[NF * NFXY];   // x faces, then y faces, of the current plane

    const int64_t blk = xcd_remap(blockIdx.x, args.nblocks);
    const int gi = find_group(args.g, args.ngroups, blk);
    const Group& g = args.g[gi];
    const int64_t local = blk - g.block0;
    const int32_t sample = (int32_t)(local / g.ntiles);
    const int32_t tile = (int32_t)(local % g.ntiles);
    if (!g.active[sample]) return;   // uniform across the workgroup

    const int32_t tx = tile % g.tiles[0];
    const int32_t ty = (tile / g.tiles[0]) % g.tiles[1];
    const int32_t tz = tile / (g.tiles[0] * g.tiles[1]);
    const int32_t x0 = tx * BX, y0 = ty * BY, z0 = tz * BZ;
    const int32_t nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const int32_t z1 = (z0 + BZ < nz) ? z0 + BZ : nz;
    const int64_t cells = g.cells;
    const int32_t plane = nx * ny;   // cells < 2^31: indices within a sample are 32-bit
    const int64_t sbase = (int64_t)sample * NF * cells;
    const double* src = g.src + sbase;
    const double* un = g.un + sbase;
    double* dst = g.dst + sbase;
    const int t = threadIdx.x;

    // this thread's column (threads past the block's columns shadow its last column and
    // store nothing)
    const int col = (t < COLS) ? t : COLS - 1;
    const int cx = col % BX, cy = col / BX;
    const bool own = (t < COLS) && (x0 + cx < nx) && (y0 + cy < ny);
    const int32_t ccol = wrap_index(y0 + cy, ny, args.bc[1]) * nx + wrap_index(x0 + cx, nx, args.bc[0]);
    const int lcore = (cy + G) * PX + (cx + G);

    // this thread's halo cell (threads t >= NH have none)
    int hpx = 0, hpy = 0;
    if (t < NH) z_halo_pos<G, BX, BY>(t, hpx, hpy);
    const int lhalo = hpy * PX + hpx;
    const int32_t chalo = wrap_index(y0 + hpy - G, ny, args.bc[1]) * nx
                        + wrap_index(x0 + hpx - G, nx, args.bc[0]);

    // column window: w[j] = cell z = k - G + 1 + j at the face above plane k
    double w[2 * G][NF];
#pragma unroll
    for (int j = 0; j < 2 * G; ++j) {
        const int32_t zc = wrap_index(z0 - G + j, nz, args.bc[2]) * plane + ccol;
#pragma unroll
        for (int q = 0; q < NF; ++q) w[j][q] = src[q * cells + zc];
    }
    double hreg[NF];
    if (t < NH) {
        const int32_t hc = z0 * plane + chalo;
#pragma unroll
        for (int q = 0; q < NF; ++q) hreg[q] = src[q * cells + hc];
    }
    double fzm[NF];   // z flux on the lower face of the current plane
    z_column_face<EQ, RECON, FLUX, NF, G>(w, g.ph, fzm);
#pragma unroll
    for (int j = 0; j + 1 < 2 * G; ++j)
#pragma unroll
        for (int q = 0; q < NF; ++q) w[j][q] = w[j + 1][q];

    const double dt = g.dt[sample];
    const double beta = args.beta;
    double m = 0.0;
    bool bad = false;

    for (int32_t k = z0; k < z1; ++k) {
        // 1. stage plane k: its own cells from the column registers, the halo from registers
        //    filled one plane ahead
        if (t < COLS) {
#pragma unroll
            for (int q = 0; q < NF; ++q) sp[q * PP + lcore] = w[G - 1][q];
        }
        if (t < NH) {
#pragma unroll
            for (int q = 0; q < NF; ++q) sp[q * PP + lhalo] = hreg[q];
        }
        // 2. request the column cell k + G, the halo of plane k + 1 and (compiled for 3
        //    wavefronts per SIMD, where the registers are there) U^n of the updated cell
        {
            const int32_t zc = wrap_index(k + G, nz, args.bc[2]) * plane + ccol;
#pragma unroll
            for (int q = 0; q < NF; ++q) w[2 * G - 1][q] = src[q * cells + zc];
        }
        if (t < NH && k + 1 < z1) {
            const int32_t hc = (k + 1) * plane + chalo;
#pragma unroll
            for (int q = 0; q < NF; ++q) hreg[q] = src[q * cells + hc];
        }
        double unr[NF];
        if (WPE <= 3 && args.use_un) {
            const int32_t cc = k * plane + ccol;
#pragma unroll
            for (int q = 0; q < NF; ++q) unr[q] = un[q * cells + cc];
        }
        __syncthreads();

        // 3. x and y faces of the plane (each axis padded to whole wavefronts)
#pragma unroll
        for (int p = 0; p < T::FPT; ++p) {
            const int pf = t + p * NT;
            if (pf < T::TOTAL) {
                double F[NF];
                const int wave_first = __builtin_amdgcn_readfirstlane(pf);
                int slot;
                if (wave_first < T::PXN) {
                    const bool ok = pf < NFX;
                    z_plane_face<EQ, RECON, FLUX, BX, BY, NT, 0>(sp, g.ph, ok ? pf : NFX - 1, F);
                    slot = ok ? pf : -1;
                } else {
                    const int l = pf - T::PXN;
                    const bool ok = l < T::NFY;
                    z_plane_face<EQ, RECON, FLUX, BX, BY, NT, 1>(sp, g.ph, ok ? l : T::NFY - 1, F);
                    slot = ok ? NFX + l : -1;
                }
                if (slot >= 0) {
#pragma unroll
                    for (int q = 0; q < NF; ++q) sf[q * NFXY + slot] = F[q];
                }
            }
        }
        // 4. the z face above plane k, in registers
        double fzp[NF];
        z_column_face<EQ, RECON, FLUX, NF, G>(w, g.ph, fzp);
        __syncthreads();

        // 5. divergence (x, y, z) and the Runge--Kutta stage combination
        if (own) {
            const int fxm = cy * (BX + 1) + cx;
            const int fym = NFX + cy * BX + cx;
            const int32_t gidx = k * plane + ccol;
            double out[NF];
#pragma unroll
            for (int q = 0; q < NF; ++q) {
                const double* F = sf + q * NFXY;
                double acc = (F[fxm + 1] - F[fxm]) * g.ph.inv_dx[0];
                acc = acc + ((F[fym + BX] - F[fym]) * g.ph.inv_dx[1]);
                acc = acc + ((fzp[q] - fzm[q]) * g.ph.inv_dx[2]);
                const double rhs = -acc;
                const double up = w[G - 1][q];
                const double u0q = args.use_un ? (WPE <= 3 ? unr[q] : un[q * cells + gidx]) : up;
                out[q] = u0q + (beta * ((up - u0q) + (dt * rhs)));
                dst[q * cells + gidx] = out[q];
            }
            if (args.last) {
                bool b;
                const double s = cell_speed<3, EQ>(out, g.ph, b);
                m = vmax(m, s);
                bad = bad || b;
            }
        }
        // 6. slide the column window up by one plane
#pragma unroll
        for (int q = 0; q < NF; ++q) fzm[q] = fzp[q];
#pragma unroll
        for (int j = 0; j + 1 < 2 * G; ++j)
#pragma unroll
            for (int q = 0; q < NF; ++q) w[j][q] = w[j + 1][q];
    }
    if (args.last)
        block_merge_speed<NT>(m, bad, &g.mbits[(tile % kSpeedSlots) * speed_pitch(g.batch) + sample],
                              &g.bad[sample]);
}

template <int EQ, int RECON, int FLUX, int BX, int BY, int BZ, int NT, int WPE>
void launch_stage_z(const StageArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL((stage_kernel_z<EQ, RECON, FLUX, BX, BY, BZ, NT, WPE>),
                       dim3((unsigned)a.nblocks), dim3(NT), 0, s, a);
}

template <int EQ, int RECON, int FLUX, int BX, int BY, int BZ, int NT, int WPE>
constexpr StageKernel make_stage_kernel_z()
{
    return StageKernel{&launch_stage_z<EQ, RECON, FLUX, BX, BY, BZ, NT, WPE>, &launch_speed<3, EQ>,
                       BX, BY, BZ, kSpeedCellsPerBlock};
}

}  // namespace fvk
