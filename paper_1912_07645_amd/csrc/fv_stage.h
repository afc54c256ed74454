// fv_stage.h -- the fused Runge--Kutta stage kernel of the finite-volume scheme and the
// wave-speed reduction kernel, as templates over (dimension, equation, reconstruction,
// numerical flux, tile shape, workgroup size).
//
// One workgroup of NT threads updates one tile of BX x BY x BZ cells of one sample:
//   1. ghost fill + load: the tile and a halo of G cells on every active axis are read from
//      HBM into LDS; periodic axes wrap, transmissive axes clamp to the edge cell, so no
//      padded copy exists in memory;
//   2. faces: every face of the tile, of every axis, is reconstructed and its numerical flux
//      computed exactly once. The faces of all axes form one list (x faces, then y, then z,
//      each axis padded to whole wavefronts), dealt to the threads in order; tile shapes are
//      chosen so the list fills the workgroup's wavefronts evenly (e.g. 16 x 15 cells have
//      255 + 256 faces for 2 x 256 lanes), so no wavefront does an extra pass for the "+1"
//      row of faces that every tile has along each axis;
//   3. divergence: each cell adds (F_+ - F_-) / dx_k in the order x, y, z (eq. 2.1);
//   4. Runge--Kutta stage: U^(s) = U^n + beta ((U^(s-1) - U^n) + dt L(U^(s-1))), written to
//      HBM; in the last stage the new state's wave speed is reduced across the workgroup
//      (wavefront shuffles, then LDS) and merged into the sample's maximum with an atomic max
//      on the bit pattern (exact and order-independent), and non-physical cells are flagged.
#pragma once

#include "fv_physics.h"

namespace fvk {

template <int RECON>
struct Ghost {
    static constexpr int value = (RECON == REC_FIRST) ? 1 : 2;
};

// Ghost-cell index map: periodic wrap or transmissive clamp. Tile loads ask for indices in
// [-G, n + B + G); a single add or subtract covers them unless the grid is smaller than the
// tile plus its halo, where the remainder is taken.
__device__ __forceinline__ int32_t wrap_index(int32_t i, int32_t n, int32_t bc)
{
    if (bc == BC_PERIODIC) {
        if (i < 0) i += n;
        else if (i >= n) i -= n;
        if ((uint32_t)i >= (uint32_t)n) {
            i %= n;
            if (i < 0) i += n;
        }
        return i;
    }
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// Ghost-cell index map of a split-buffer subdomain along one axis (array coordinates): an
// axis whose ghosts are stored in the array (halo) reads them there, clamped to the array (a
// ragged last tile reaches past the halo only for cells it does not update); any other axis
// wraps or clamps as on a whole grid.
__device__ __forceinline__ int32_t halo_index(int32_t i, int32_t n, int32_t bc, int32_t off,
                                              int32_t pn, bool halo)
{
    if (halo) {
        const int32_t a = i + off;
        return a < 0 ? 0 : (a >= pn ? pn - 1 : a);
    }
    return wrap_index(i, n, bc) + off;
}

// Workgroups are dealt round-robin to the 8 XCDs; remap so that each XCD receives a
// contiguous range of tiles and halo re-reads of neighbouring tiles hit its own L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nblocks)
{
    const int64_t full = (nblocks / 8) * 8;
    if (b >= full) return b;
    return (b % 8) * (full / 8) + (b / 8);
}

template <int DIM, int EQ, int RECON, int BX, int BY, int BZ, int NT>
struct StageTile {
    static constexpr int NF = NumFields<DIM, EQ>::value;
    static constexpr int G = Ghost<RECON>::value;
    static constexpr int PX = BX + 2 * G;
    static constexpr int PY = (DIM >= 2) ? BY + 2 * G : 1;
    static constexpr int PZ = (DIM >= 3) ? BZ + 2 * G : 1;
    static constexpr int PCELLS = PX * PY * PZ;
    static constexpr int CELLS = BX * BY * BZ;
    static constexpr int CPT = (CELLS + NT - 1) / NT;   // cells per thread
    static constexpr int NFX = (BX + 1) * BY * BZ;       // faces normal to x
    static constexpr int NFY = (DIM >= 2) ? BX * (BY + 1) * BZ : 0;
    static constexpr int NFZ = (DIM >= 3) ? BX * BY * (BZ + 1) : 0;
    static constexpr int NFACES = NFX + NFY + NFZ;
    static_assert(NT % 64 == 0, "whole wavefronts");
    static_assert(DIM >= 2 || (BY == 1 && BZ == 1), "1D tiles are rows");
    static_assert(DIM >= 3 || BZ == 1, "2D tiles are flat");
};

// LDS layouts of the haloed state tile. LAY_FIELD: one block per conserved field,
// [q][z][y][x]. LAY_ROW: the fields interleaved row by row, [z][y][q][x], so that the halo
// rows of the y axis are whole contiguous blocks at both ends of the tile.
enum { LAY_FIELD = 0, LAY_ROW = 1 };

template <int NF, int PX, int PY, int PZ, int LAY>
struct TileLayout {
    static constexpr int QS = (LAY == LAY_FIELD) ? PX * PY * PZ : PX;   // field stride
    static constexpr int RS = (LAY == LAY_FIELD) ? PX : NF * PX;        // y stride
    static constexpr int PS = RS * PY;                                  // z stride
};

// One face with normal axis ND (compile-time): reconstruction from the LDS tile and the
// numerical flux into F.
template <int DIM, int EQ, int RECON, int FLUX, int BX, int BY, int BZ, int NT, int ND,
          int LAY = LAY_FIELD>
__device__ __forceinline__ void one_face(const double* su, const Phys& ph, int l, double* F)
{
    using T = StageTile<DIM, EQ, RECON, BX, BY, BZ, NT>;
    using TL = TileLayout<T::NF, T::PX, T::PY, T::PZ, LAY>;
    constexpr int NF = T::NF, G = T::G;
    constexpr int GY = (DIM >= 2) ? G : 0, GZ = (DIM >= 3) ? G : 0;
    constexpr int EX = BX + (ND == 0), EY = BY + (ND == 1);
    constexpr int STRIDE = (ND == 0) ? 1 : ((ND == 1) ? TL::RS : TL::PS);
    const int fx = l % EX;
    const int fy = (l / EX) % EY;
    const int fz = l / (EX * EY);
    // LDS index of the cell on the right of the face (the face is its "minus" side)
    const int c = (fz + GZ) * TL::PS + (fy + GY) * TL::RS + (fx + G);
    if constexpr (FLUX == FLUX_EC4) {
        static_assert(RECON == REC_CELLS4, "the fourth-order EC flux reads cell values");
        double A[NF], B[NF], C[NF], D[NF];
#pragma unroll
        for (int q = 0; q < NF; ++q) {
            const double* s = su + q * TL::QS + c;
            A[q] = s[-2 * STRIDE];
            B[q] = s[-STRIDE];
            C[q] = s[0];
            D[q] = s[STRIDE];
        }
        ec4_face<DIM, EQ>(A, B, C, D, ND, F, ph);
    } else {
        double UL[NF], UR[NF];
#pragma unroll
        for (int q = 0; q < NF; ++q) {
            const double* s = su + q * TL::QS + c;
            if (RECON == REC_FIRST) {
                reconstruct<RECON>(0.0, s[-STRIDE], s[0], 0.0, UL[q], UR[q]);
            } else {
                reconstruct<RECON>(s[-2 * STRIDE], s[-STRIDE], s[0], s[STRIDE], UL[q], UR[q]);
            }
        }
        numflux<DIM, EQ, FLUX>(UL, UR, ND, F, ph);
    }
}

// Padded face list: each axis's faces rounded up to whole wavefronts, so the faces a
// wavefront takes in one pass share one axis (wave-uniform, a compile-time face routine).
template <int DIM, int EQ, int RECON, int BX, int BY, int BZ, int NT>
struct FaceList {
    using T = StageTile<DIM, EQ, RECON, BX, BY, BZ, NT>;
    static constexpr int PXN = (T::NFX + 63) / 64 * 64;
    static constexpr int PYN = (T::NFY + 63) / 64 * 64;
    static constexpr int PZN = (T::NFZ + 63) / 64 * 64;
    static constexpr int TOTAL = PXN + PYN + PZN;
    static constexpr int FPT = (TOTAL + NT - 1) / NT;   // faces per thread
};

// LDS plan of HOLD = 2 (2D, LAY_ROW tile): the y faces are computed first. Once every
// thread has read the tile, the y halo rows (the first and last G rows, contiguous in
// LAY_ROW) are dead; the x fluxes, [q][face], are written from the start of the low halo
// rows, continue at the start of the high halo rows and run on past the tile, and the y
// fluxes, [q][face], follow. The workgroup needs the tile plus its faces minus those rows.
template <int DIM, int EQ, int RECON, int BX, int BY, int BZ, int NT>
struct SplitFaces {
    using T = StageTile<DIM, EQ, RECON, BX, BY, BZ, NT>;
    static constexpr int NF = T::NF, NFX = T::NFX, NFY = T::NFY;
    static constexpr int SU = NF * T::PCELLS;
    static constexpr int LOW = T::G * NF * T::PX;            // low halo rows: [0, LOW)
    static constexpr int HIGH = (BY + T::G) * NF * T::PX;    // high halo rows: [HIGH, SU)
    static constexpr int YB = HIGH + NF * NFX - LOW;         // first y flux
    static constexpr int LDS = YB + NF * NFY;
    // LDS index of x flux j = q * NFX + face
    __device__ static __forceinline__ int x_at(int j) { return j < LOW ? j : j + (HIGH - LOW); }
    // the same for field q, with the branch resolved at compile time where q decides it
    __device__ static __forceinline__ int x_at(int q, int face)
    {
        const int j = q * NFX + face;
        if ((q + 1) * NFX <= LOW) return j;
        if (q * NFX >= LOW) return j + (HIGH - LOW);
        return x_at(j);
    }
};

// Face pf of the padded list: F gets its flux, *slot its index in the unpadded list sf[q][f]
// (-1 for padding; padding lanes recompute a valid face and store nothing).
template <int DIM, int EQ, int RECON, int FLUX, int BX, int BY, int BZ, int NT>
__device__ __forceinline__ void list_face(const double* su, const Phys& ph, int pf, double* F,
                                          int* slot)
{
    using T = StageTile<DIM, EQ, RECON, BX, BY, BZ, NT>;
    using L = FaceList<DIM, EQ, RECON, BX, BY, BZ, NT>;
    constexpr int NFX = T::NFX, NFY = T::NFY, NFZ = T::NFZ;
    const int wave_first = __builtin_amdgcn_readfirstlane(pf);  // same axis for the wave
    if (wave_first < L::PXN) {
        const int l = pf;
        const bool ok = l < NFX;
        one_face<DIM, EQ, RECON, FLUX, BX, BY, BZ, NT, 0>(su, ph, ok ? l : NFX - 1, F);
        *slot = ok ? l : -1;
    } else if (DIM >= 2 && wave_first < L::PXN + L::PYN) {
        const int l = pf - L::PXN;
        const bool ok = l < NFY;
        one_face<DIM, EQ, RECON, FLUX, BX, BY, BZ, NT, (DIM >= 2 ? 1 : 0)>(su, ph, ok ? l : NFY - 1, F);
        *slot = ok ? NFX + l : -1;
    } else {
        const int l = pf - L::PXN - L::PYN;
        const bool ok = DIM >= 3 && l < NFZ;
        one_face<DIM, EQ, RECON, FLUX, BX, BY, BZ, NT, (DIM >= 3 ? 2 : 0)>(su, ph, ok ? l : (NFZ > 0 ? NFZ - 1 : 0), F);
        *slot = ok ? NFX + NFY + l : -1;
    }
}

// All faces of the tile into sf[q][face] (x faces, then y faces, then z faces).
// HOLD = 0: each flux goes to its own LDS face buffer as soon as it is computed.
// HOLD = 1: each thread keeps its fluxes in registers until every thread has finished
// reading the state tile, then they are written over it (sf aliases su): the workgroup
// needs max(state tile, faces) of LDS instead of their sum, so more workgroups fit a CU.
// HOLD = 2: y faces, then x faces written over the dead y halo rows (SplitFaces).
template <int DIM, int EQ, int RECON, int FLUX, int BX, int BY, int BZ, int NT, int HOLD>
__device__ __forceinline__ void tile_faces(const double* su, double* sf, const Phys& ph)
{
    using T = StageTile<DIM, EQ, RECON, BX, BY, BZ, NT>;
    using L = FaceList<DIM, EQ, RECON, BX, BY, BZ, NT>;
    constexpr int NF = T::NF, NFACES = T::NFACES;
    if constexpr (HOLD == 2) {
        static_assert(DIM == 2, "split faces are for 2D tiles");
        using S = SplitFaces<DIM, EQ, RECON, BX, BY, BZ, NT>;
        constexpr int NFX = T::NFX, NFY = T::NFY;
        static_assert(NF * NFX >= S::LOW && S::YB >= S::SU, "x fluxes cover the low halo rows");
        for (int pf = threadIdx.x; pf < L::PYN; pf += NT) {
            double F[NF];
            one_face<DIM, EQ, RECON, FLUX, BX, BY, BZ, NT, 1, LAY_ROW>(su, ph, pf < NFY ? pf : NFY - 1, F);
            if (pf < NFY) {
#pragma unroll
                for (int q = 0; q < NF; ++q) sf[S::YB + q * NFY + pf] = F[q];
            }
        }
        __syncthreads();   // the y halo rows are dead from here on
        for (int pf = threadIdx.x; pf < L::PXN; pf += NT) {
            double F[NF];
            one_face<DIM, EQ, RECON, FLUX, BX, BY, BZ, NT, 0, LAY_ROW>(su, ph, pf < NFX ? pf : NFX - 1, F);
            if (pf < NFX) {
#pragma unroll
                for (int q = 0; q < NF; ++q) sf[S::x_at(q, pf)] = F[q];
            }
        }
    } else if constexpr (!HOLD) {
        for (int pf = threadIdx.x; pf < L::TOTAL; pf += NT) {
            double F[NF];
            int slot;
            list_face<DIM, EQ, RECON, FLUX, BX, BY, BZ, NT>(su, ph, pf, F, &slot);
            if (slot >= 0) {
#pragma unroll
                for (int q = 0; q < NF; ++q) sf[q * NFACES + slot] = F[q];
            }
        }
    } else {
        double F[L::FPT][NF];
        int slot[L::FPT];
#pragma unroll
        for (int k = 0; k < L::FPT; ++k) {
            const int pf = threadIdx.x + k * NT;
            slot[k] = -1;
            if (pf < L::TOTAL) list_face<DIM, EQ, RECON, FLUX, BX, BY, BZ, NT>(su, ph, pf, F[k], &slot[k]);
        }
        __syncthreads();   // the state tile is dead from here on
#pragma unroll
        for (int k = 0; k < L::FPT; ++k) {
            if (slot[k] >= 0) {
#pragma unroll
                for (int q = 0; q < NF; ++q) sf[q * NFACES + slot[k]] = F[k][q];
            }
        }
    }
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = vmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Reduce (m, bad) across the workgroup and merge into the sample's words.
template <int NT>
__device__ __forceinline__ void block_merge_speed(double m, bool bad, unsigned long long* mbits,
                                                  int32_t* badflag)
{
    __shared__ double red[NT / 64];
    __shared__ int redbad;
    if (threadIdx.x == 0) redbad = 0;
    __syncthreads();
    m = wave_max(m);
    if (bad) atomicOr(&redbad, 1);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = red[0];
#pragma unroll
        for (int w = 1; w < NT / 64; ++w) r = vmax(r, red[w]);
        atomicMax(mbits, (unsigned long long)__double_as_longlong(r));
        if (redbad) atomicOr(badflag, 1);
    }
}

__device__ __forceinline__ int find_group(const Group* g, int ngroups, int64_t block)
{
    int gi = 0;
#pragma unroll
    for (int i = 1; i < kMaxGroups; ++i)
        if (i < ngroups && block >= g[i].block0) gi = i;
    return gi;
}

// Fewest waves per SIMD the register allocation must leave room for: 6 for the LDS-held tile
// plans; the Euler Godunov flux (a Newton iteration with logarithms and exponentials) needs
// 116-148 registers and would spill under the 80 that 6 waves leave, so it is allowed 2.
template <int EQ, int FLUX, int HOLD>
constexpr int stage_min_waves() { return (FLUX == FLUX_GODUNOV && EQ == EQ_EULER) ? 2 : (HOLD ? 6 : 1); }

// HALO = 1: the split-buffer form. Arrays are subdomains with stored ghost layers on the axes
// of g.hmask (Group), and the launch covers the box of tiles g.tlo + [0, g.tcnt) of each group;
// the arithmetic per cell is the same as for the whole grid.
template <int DIM, int EQ, int RECON, int FLUX, int BX, int BY, int BZ, int NT, int HOLD,
          int HALO = 0>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(stage_min_waves<EQ, FLUX, HOLD>(), 8)))
stage_kernel(const StageArgs args)
{
    using T = StageTile<DIM, EQ, RECON, BX, BY, BZ, NT>;
    constexpr int NF = T::NF, G = T::G, PX = T::PX, PY = T::PY;
    constexpr int PCELLS = T::PCELLS, CPT = T::CPT, CELLS = T::CELLS;
    constexpr int NFX = T::NFX, NFY = T::NFY, NFACES = T::NFACES;
    constexpr int GY = (DIM >= 2) ? G : 0, GZ = (DIM >= 3) ? G : 0;
    constexpr int SU = NF * PCELLS, SF = NF * NFACES;
    constexpr int LAY = (HOLD == 2) ? LAY_ROW : LAY_FIELD;
    using TL = TileLayout<NF, PX, PY, T::PZ, LAY>;
    using S = SplitFaces<DIM, EQ, RECON, BX, BY, BZ, NT>;
    constexpr int LDS = (HOLD == 1) ? (SU > SF ? SU : SF) : ((HOLD == 2) ? S::LDS : SU + SF);
    __shared__ double lds[LDS];
    double* su = lds;
    double* sf = (HOLD != 0) ? lds : lds + SU;

    const int64_t blk = xcd_remap(blockIdx.x, args.nblocks);
    const int gi = find_group(args.g, args.ngroups, blk);
    const Group& g = args.g[gi];
    const int64_t local = blk - g.block0;
    const int32_t sample = (int32_t)(local / g.ntiles);
    const int32_t tile = (int32_t)(local % g.ntiles);
    if (!g.active[sample]) return;   // uniform across the workgroup

    int32_t tx, ty, tz;
    if constexpr (HALO) {
        tx = g.tlo[0] + tile % g.tcnt[0];
        ty = g.tlo[1] + (tile / g.tcnt[0]) % g.tcnt[1];
        tz = g.tlo[2] + tile / (g.tcnt[0] * g.tcnt[1]);
    } else {
        tx = tile % g.tiles[0];
        ty = (tile / g.tiles[0]) % g.tiles[1];
        tz = tile / (g.tiles[0] * g.tiles[1]);
    }
    const int32_t x0 = tx * BX, y0 = ty * BY, z0 = tz * BZ;
    const int32_t nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const int64_t sbase = (int64_t)sample * NF * g.cells;
    const double* src = g.src + sbase;

    // the thread's cells: cell k is tile cell threadIdx.x + k * NT
    int32_t cell_g[CPT];   // index in the sample
    bool cell_ok[CPT];     // inside the tile and the grid
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
        const int c = threadIdx.x + k * NT;
        const int cx = c % BX;
        const int cy = (c / BX) % BY;
        const int cz = c / (BX * BY);
        const int32_t gx = x0 + cx, gy = y0 + cy, gz = z0 + cz;
        cell_ok[k] = c < CELLS && gx < nx && gy < ny && gz < nz;
        if constexpr (HALO)
            cell_g[k] = ((gz + g.off[2]) * g.pn[1] + (gy + g.off[1])) * g.pn[0] + (gx + g.off[0]);
        else
            cell_g[k] = (gz * ny + gy) * nx + gx;   // cells < 2^31
    }
    const double* un = g.un + sbase;
    double unr[CPT][NF];

    // 1. ghost fill + load of the haloed tile into LDS: every load of the thread is issued
    //    before the first LDS store, so the tile costs one memory round trip
    {
        constexpr int LPT = (PCELLS + NT - 1) / NT;
        double v[LPT][NF];
#pragma unroll
        for (int k = 0; k < LPT; ++k) {
            const int e = threadIdx.x + k * NT;
            if ((k + 1) * NT <= PCELLS || e < PCELLS) {
                const int px = e % PX;
                const int py = (e / PX) % PY;
                const int pz = e / (PX * PY);
                int32_t gidx;
                if constexpr (HALO) {
                    const int32_t ax = halo_index(x0 + px - G, nx, args.bc[0], g.off[0], g.pn[0], g.hmask & 1);
                    const int32_t ay = (DIM >= 2) ? halo_index(y0 + py - G, ny, args.bc[1], g.off[1], g.pn[1], g.hmask & 2) : 0;
                    const int32_t az = (DIM >= 3) ? halo_index(z0 + pz - G, nz, args.bc[2], g.off[2], g.pn[2], g.hmask & 4) : 0;
                    gidx = (az * g.pn[1] + ay) * g.pn[0] + ax;
                } else {
                    const int32_t gx = wrap_index(x0 + px - G, nx, args.bc[0]);
                    const int32_t gy = (DIM >= 2) ? wrap_index(y0 + py - G, ny, args.bc[1]) : 0;
                    const int32_t gz = (DIM >= 3) ? wrap_index(z0 + pz - G, nz, args.bc[2]) : 0;
                    gidx = (gz * ny + gy) * nx + gx;   // cells < 2^31
                }
#pragma unroll
                for (int q = 0; q < NF; ++q) v[k][q] = src[q * g.cells + gidx];
            }
        }
        // U^n of the thread's cells (stages >= 2), requested with the tile so that its
        // latency hides behind the faces (not where the fluxes are held in registers: there
        // the extra registers cost more than the wait)
        if (HOLD != 1 && args.use_un) {
#pragma unroll
            for (int k = 0; k < CPT; ++k) {
                if (cell_ok[k]) {
#pragma unroll
                    for (int q = 0; q < NF; ++q) unr[k][q] = un[q * g.cells + cell_g[k]];
                }
            }
        }
#pragma unroll
        for (int k = 0; k < LPT; ++k) {
            const int e = threadIdx.x + k * NT;
            if ((k + 1) * NT <= PCELLS || e < PCELLS) {
                const int px = e % PX;
                const int row = e / PX;   // z * PY + y
#pragma unroll
                for (int q = 0; q < NF; ++q)
                    su[(LAY == LAY_FIELD) ? q * PCELLS + e : row * TL::RS + q * TL::QS + px] = v[k][q];
            }
        }
    }
    __syncthreads();

    // 2. every face of the tile, once
    tile_faces<DIM, EQ, RECON, FLUX, BX, BY, BZ, NT, HOLD>(su, sf, g.ph);
    __syncthreads();

    // 3 + 4. divergence and Runge--Kutta stage combination
    const double dt = g.dt[sample];
    const double beta = args.beta;
    double m = 0.0;
    bool bad = false;
    double* dst = g.dst + sbase;
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
        if (!cell_ok[k]) continue;
        const int c = threadIdx.x + k * NT;
        const int cx = c % BX;
        const int cy = (c / BX) % BY;
        const int cz = c / (BX * BY);
        const int32_t gidx = cell_g[k];
        const int lc = (cz + GZ) * TL::PS + (cy + GY) * TL::RS + (cx + G);
        const int fxm = (cz * BY + cy) * (BX + 1) + cx;
        const int fym = NFX + (cz * (BY + 1) + cy) * BX + cx;
        const int fzm = NFX + NFY + (cz * BY + cy) * BX + cx;
        double out[NF];
#pragma unroll
        for (int q = 0; q < NF; ++q) {
            double acc;
            if constexpr (HOLD == 2) {
                const int fyl = cy * BX + cx;
                const double* Fy = sf + S::YB + q * NFY;
                acc = (sf[S::x_at(q, fxm + 1)] - sf[S::x_at(q, fxm)]) * g.ph.inv_dx[0];
                acc = acc + ((Fy[fyl + BX] - Fy[fyl]) * g.ph.inv_dx[1]);
            } else {
                const double* F = sf + q * NFACES;
                acc = (F[fxm + 1] - F[fxm]) * g.ph.inv_dx[0];
                if (DIM >= 2) acc = acc + ((F[fym + BX] - F[fym]) * g.ph.inv_dx[1]);
                if (DIM >= 3) acc = acc + ((F[fzm + BX * BY] - F[fzm]) * g.ph.inv_dx[2]);
            }
            const double rhs = -acc;
            const double up = (HOLD == 1) ? src[q * g.cells + gidx] : su[q * TL::QS + lc];
            const double u0 = args.use_un ? ((HOLD == 1) ? un[q * g.cells + gidx] : unr[k][q]) : up;
            out[q] = u0 + (beta * ((up - u0) + (dt * rhs)));
            dst[q * g.cells + gidx] = out[q];
        }
        if (args.last) {
            bool b;
            const double s = cell_speed<DIM, EQ>(out, g.ph, b);
            m = vmax(m, s);
            bad = bad || b;
        }
    }
    if (args.last)
        block_merge_speed<NT>(m, bad, &g.mbits[(tile % kSpeedSlots) * speed_pitch(g.batch) + sample],
                              &g.bad[sample]);
}

// Wave speed and physicality of a state, without update (the step-0 reduction). HALO = 1:
// over the owned cells of split-buffer subdomains (Group pn, off).
template <int DIM, int EQ, int HALO = 0>
__global__ void __launch_bounds__(kThreads)
speed_kernel(const SpeedArgs args, int cells_per_block)
{
    constexpr int NF = NumFields<DIM, EQ>::value;
    const int64_t blk = blockIdx.x;
    const int gi = find_group(args.g, args.ngroups, blk);
    const Group& g = args.g[gi];
    const int64_t local = blk - g.block0;
    const int64_t owned = HALO ? (int64_t)g.n[0] * g.n[1] * g.n[2] : g.cells;
    const int64_t per_sample = (owned + cells_per_block - 1) / cells_per_block;
    const int32_t sample = (int32_t)(local / per_sample);
    const int64_t c0 = (local % per_sample) * cells_per_block;
    if (!g.active[sample]) return;
    const double* src = g.src + (int64_t)sample * NF * g.cells;
    double m = 0.0;
    bool bad = false;
    for (int64_t c = c0 + threadIdx.x; c < c0 + cells_per_block && c < owned; c += kThreads) {
        int64_t a = c;
        if constexpr (HALO) {
            const int64_t x = c % g.n[0], y = (c / g.n[0]) % g.n[1], z = c / ((int64_t)g.n[0] * g.n[1]);
            a = ((z + g.off[2]) * g.pn[1] + (y + g.off[1])) * g.pn[0] + (x + g.off[0]);
        }
        double U[NF];
#pragma unroll
        for (int q = 0; q < NF; ++q) U[q] = src[q * g.cells + a];
        bool b;
        const double s = cell_speed<DIM, EQ>(U, g.ph, b);
        m = vmax(m, s);
        bad = bad || b;
    }
    block_merge_speed<kThreads>(m, bad,
                                &g.mbits[((local % per_sample) % kSpeedSlots) * speed_pitch(g.batch) + sample],
                                &g.bad[sample]);
}

template <int DIM, int EQ, int RECON, int FLUX, int BX, int BY, int BZ, int NT, int HOLD,
          int HALO = 0>
void launch_stage(const StageArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL((stage_kernel<DIM, EQ, RECON, FLUX, BX, BY, BZ, NT, HOLD, HALO>),
                       dim3((unsigned)a.nblocks), dim3(NT), 0, s, a);
}

constexpr int kSpeedCellsPerBlock = 4096;

template <int DIM, int EQ, int HALO = 0>
void launch_speed(const SpeedArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL((speed_kernel<DIM, EQ, HALO>), dim3((unsigned)a.nblocks), dim3(kThreads), 0,
                       s, a, kSpeedCellsPerBlock);
}

// Default LDS plan: split faces in 2D, fluxes held in registers otherwise.
template <int DIM, int EQ, int RECON, int FLUX, int BX, int BY, int BZ, int NT,
          int HOLD = (DIM == 2) ? 2 : 1, int HALO = 0>
constexpr StageKernel make_stage_kernel()
{
    return StageKernel{&launch_stage<DIM, EQ, RECON, FLUX, BX, BY, BZ, NT, HOLD, HALO>,
                       &launch_speed<DIM, EQ, HALO>, BX, BY, BZ, kSpeedCellsPerBlock};
}

}  // namespace fvk
