// fv_stats.hip -- on-device Monte Carlo statistics (Section 2.2): per-cell mean and
// variance of the quantities over samples (Welford, samples in index order) and the
// second-order two-point structure function S_q(h) of every sample, averaged over samples.
//
// Quantities: Euler (rho, u_1..u_dim, E) with u_k = m_k * (1 / rho); scalar: the field.
#include "fv_stats.h"

#include <algorithm>

namespace fvk {

// Per-cell Welford update over the samples of one batch, in sample order. A workgroup covers
// 64 cells with one wavefront per quantity (64 NF threads): each thread keeps the running
// moments of one (cell, quantity) in registers, so a batch has NF times as many wavefronts as
// cells / 64. The loads of the next kWelfordDepth samples are issued before the current ones
// are processed, so each thread has that many samples' loads in flight. With qout, the
// quantities are also written there ([sample][quantity][cells]) for the structure functions.
// KIND: 0 the field itself; 1 Euler (the momenta divided by rho); 2 shallow water (the
// momenta divided by h); 3 ideal MHD (the three momenta divided by rho). The divisor is field
// 0. SHARE: its own wavefront, which loads it anyway, passes each group of samples' values to
// the other wavefronts through LDS (two buffers, one barrier per group), so every field of a
// sample is read from memory once; otherwise each dividing wavefront loads field 0 itself.
// The launch without qout shares (fewer bytes: 400 us against 472 us for 1024 samples of 256^2
// Euler); the one that writes the quantities does not (there the barrier costs more than the
// re-reads: 251 us against 216 us for 256 samples).
constexpr int kWelfordDepth = 8;

template <int NF, int KIND, bool SHARE>
__global__ void __launch_bounds__(512)
welford_kernel(const double* __restrict__ state, int64_t cells, int32_t batch, int64_t count0,
               double* __restrict__ mean, double* __restrict__ m2, double* __restrict__ qout)
{
    static_assert(!SHARE || KIND != 0, "only quantities divided by field 0 share it");
    constexpr int D = kWelfordDepth;
    __shared__ double f0[SHARE ? 2 * D * 64 : 1];   // [group parity][sample][cell]
    const int q = threadIdx.x >> 6;   // the wavefront's quantity
    const int lane = threadIdx.x & 63;
    const int64_t c = (int64_t)blockIdx.x * 64 + lane;
    const bool live = c < cells;      // lanes past the last cell only take part in barriers
    if (!SHARE && !live) return;      // no barrier without SHARE: such lanes leave at once
    constexpr int DIV_END = (KIND == 1) ? NF - 1 : ((KIND == 3) ? 4 : NF);
    const bool div = KIND != 0 && q >= 1 && q < DIV_END;   // uniform across the wavefront
    const int64_t per = (int64_t)NF * cells;
    const double* F = state + q * cells + (live ? c : 0);
    const double* R = state + (live ? c : 0);
    constexpr bool LOADR = KIND != 0 && !SHARE;   // dividing wavefronts load field 0 themselves
    double mu = live ? mean[q * cells + c] : 0.0, s2 = live ? m2[q * cells + c] : 0.0;
    double xc[D], rc[LOADR ? D : 1];
#pragma unroll
    for (int i = 0; i < D; ++i) {
        xc[i] = (live && i < batch) ? F[i * per] : 0.0;
        if constexpr (LOADR) rc[i] = (div && live && i < batch) ? R[i * per] : 1.0;
    }
    for (int32_t b0 = 0, g = 0; b0 < batch; b0 += D, ++g) {
        double xn[D], rn[LOADR ? D : 1];
#pragma unroll
        for (int i = 0; i < D; ++i) {   // the next group's loads, before this group's work
            const int32_t b = b0 + D + i;
            xn[i] = (live && b < batch) ? F[b * per] : 0.0;
            if constexpr (LOADR) rn[i] = (div && live && b < batch) ? R[b * per] : 1.0;
        }
        double* sh = f0 + (SHARE ? (g & 1) * D * 64 : 0);
        if constexpr (SHARE) {
            // the buffer written here was last read before the previous group's barrier
            if (q == 0) {
#pragma unroll
                for (int i = 0; i < D; ++i) sh[i * 64 + lane] = xc[i];
            }
            __syncthreads();
        }
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const int32_t b = b0 + i;
            if (live && b < batch) {
                double x = xc[i];
                if constexpr (SHARE) {
                    if (div) x = xc[i] * (1.0 / sh[i * 64 + lane]);
                } else if constexpr (LOADR) {
                    if (div) x = xc[i] * (1.0 / rc[i]);
                }
                if (qout) qout[b * per + q * cells + c] = x;
                const double n = (double)(count0 + b + 1);
                const double delta = x - mu;
                mu = mu + (delta / n);
                s2 = s2 + (delta * (x - mu));
            }
        }
#pragma unroll
        for (int i = 0; i < D; ++i) {
            xc[i] = xn[i];
            if constexpr (LOADR) rc[i] = rn[i];
        }
    }
    if (live) {
        mean[q * cells + c] = mu;
        m2[q * cells + c] = s2;
    }
}

// Structure-function partial sums. Every line of cells along every axis is cut into segments
// of kSfSeg cells; a thread takes kSfSegsPerThread segments and accumulates, kSfLag lags at a
// time, sum_cells (q(x + h e) - q(x))^2 over their cells: the segment's values and the window
// q(x0 + h0 .. x0 + h0 + kSfSeg + kSfLag - 2) are loaded first (no load waits on arithmetic),
// then the kSfSeg x kSfLag terms run with compile-time indices. Segments along y and z are
// dealt so that neighbouring lanes take neighbouring lines (coalesced loads); along x,
// neighbouring lanes take neighbouring segments of a row. The chunk's lags are summed over
// the workgroup in a fixed order through LDS (per lag: 16 runs of 16 threads, then the 16
// run sums) into one partial per workgroup. Grid: (workgroups per field, quantity, sample).
constexpr int kSfSeg = 16;
constexpr int kSfLag = 16;
constexpr int kSfWin = kSfSeg + kSfLag - 1;
constexpr int kSfThreads = 256;
constexpr int kSfSegsPerThread = 2;
constexpr int kSfRowLoads = (40 * 1024 / 8 + kSfThreads - 1) / kSfThreads;   // 20

struct SfGeom {
    int32_t n[3];          // grid
    int32_t dim;
    int64_t lines[3];      // lines along axis d: cells / n[d]
    int64_t segs[3];       // segments per line along axis d
    int64_t items[4];      // first segment of axis d (items[dim] = total)
};

// Segments of the axes first..dim-1 (the x axis may be taken by the row kernel below).
static SfGeom sf_geom(int32_t dim, const int32_t n[3], int first)
{
    SfGeom g{};
    g.dim = dim;
    const int64_t cells = (int64_t)n[0] * n[1] * n[2];
    int64_t acc = 0;
    for (int d = 0; d < 3; ++d) {
        g.n[d] = n[d];
        g.lines[d] = cells / n[d];
        g.segs[d] = (n[d] + kSfSeg - 1) / kSfSeg;
        g.items[d] = acc;
        if (d >= first && d < dim) acc += g.lines[d] * g.segs[d];
    }
    g.items[dim] = acc;
    for (int d = dim + 1; d < 4; ++d) g.items[d] = acc;
    return g;
}

// Segment `item`: first cell base + x0 * stride along a line of nd cells, len cells in it.
struct SfSeg {
    int64_t base, stride;
    int32_t x0, nd, len;
};

__device__ __forceinline__ SfSeg sf_segment(const SfGeom& geo, int64_t item)
{
    SfSeg sg;
    if (item >= geo.items[geo.dim]) {   // no segment: nothing is read or added
        sg.base = 0; sg.stride = 1; sg.x0 = 0; sg.nd = 1; sg.len = 0;
        return sg;
    }
    int d = 0;
    if (item >= geo.items[1]) d = 1;
    if (item >= geo.items[2]) d = 2;
    const int64_t local = item - geo.items[d];
    sg.nd = geo.n[d];
    if (d == 0) {   // lanes along a row: item = line * segs + segment
        const int64_t line = local / geo.segs[0];
        sg.x0 = (int32_t)(local % geo.segs[0]) * kSfSeg;
        sg.base = line * geo.n[0];
        sg.stride = 1;
    } else {        // lanes across lines: item = segment * lines + line
        const int64_t line = local % geo.lines[d];
        sg.x0 = (int32_t)(local / geo.lines[d]) * kSfSeg;
        if (d == 1) {
            const int64_t xi = line % geo.n[0], zi = line / geo.n[0];
            sg.base = zi * geo.n[0] * geo.n[1] + xi;
            sg.stride = geo.n[0];
        } else {
            sg.base = line;
            sg.stride = (int64_t)geo.n[0] * geo.n[1];
        }
    }
    sg.len = (sg.nd - sg.x0 < kSfSeg) ? sg.nd - sg.x0 : kSfSeg;
    return sg;
}

// The workgroup's sums of the chunk's kSfLag lags, stored as partial number blk_index of lag
// h0 + l of the field whose partials start at out (out[(h - 1) * nblk + blk]). Fixed order:
// within a wavefront a transposing butterfly over lane bits 5, 4, 3, 2 halves the lags a lane
// holds at each step (the lane keeps the half its bit selects and adds the partner's copy of
// it), so that lane i then holds lag i / 4 summed over 16 lanes; bits 1 and 0 finish the sums.
// The wavefronts' sums meet in LDS (wsum[2][waves][kSfLag], alternate halves on alternate
// chunks, so one barrier per chunk suffices) and are added in wavefront order.
static_assert(kSfLag == 16 && kSfThreads % 64 == 0, "four halving steps over lane bits 5..2");
constexpr int kSfWaves = kSfThreads / 64;

__device__ __forceinline__ void sf_block_store(const double (&acc)[kSfLag], double* wsum,
                                               int chunk, int h0, int max_h, double* out,
                                               int64_t nblk, int64_t blk_index)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double v8[8], v4[4], v2[2];
    const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8, b2 = lane & 4;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const double keep = b5 ? acc[8 + k] : acc[k];
        const double give = b5 ? acc[k] : acc[8 + k];
        v8[k] = keep + __shfl_xor(give, 32);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double keep = b4 ? v8[4 + k] : v8[k];
        const double give = b4 ? v8[k] : v8[4 + k];
        v4[k] = keep + __shfl_xor(give, 16);
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const double keep = b3 ? v4[2 + k] : v4[k];
        const double give = b3 ? v4[k] : v4[2 + k];
        v2[k] = keep + __shfl_xor(give, 8);
    }
    double v = (b2 ? v2[1] : v2[0]) + __shfl_xor(b2 ? v2[0] : v2[1], 4);
    v = v + __shfl_xor(v, 2);     // a + b and b + a are the same double
    v = v + __shfl_xor(v, 1);
    double* ws = wsum + (chunk & 1) * (kSfWaves * kSfLag);
    if ((lane & 3) == 0) ws[wave * kSfLag + (lane >> 2)] = v;
    __syncthreads();
    const int h = h0 + (int)threadIdx.x;
    if (threadIdx.x < kSfLag && h <= max_h) {
        double t = ws[threadIdx.x];
#pragma unroll
        for (int w = 1; w < kSfWaves; ++w) t = t + ws[w * kSfLag + threadIdx.x];
        out[(int64_t)(h - 1) * nblk + blk_index] = t;
    }
}

// The sums along the lines of one segment: acc[l] += sum_{r < len} (w[r + l] - v0[r])^2, each
// lag's terms in cell order.
__device__ __forceinline__ void sf_segment_terms(const double (&v0)[kSfSeg],
                                                 const double (&w)[kSfWin], int len,
                                                 double (&acc)[kSfLag])
{
#pragma unroll
    for (int r = 0; r < kSfSeg; ++r) {
        if (r < len) {
#pragma unroll
            for (int l = 0; l < kSfLag; ++l) {
                const double df = w[r + l] - v0[r];
                acc[l] = __builtin_fma(df, df, acc[l]);
            }
        }
    }
}

// Lines along y and z (and x when its rows do not fit the row kernel): segments read from
// memory, neighbouring lanes on neighbouring lines (coalesced). Partials blk_off + blk.
__global__ void __launch_bounds__(kSfThreads)
sf_partial_kernel(const double* __restrict__ q, const SfGeom geo, int32_t nq, int32_t max_h,
                  int32_t nblk, int32_t blk_off, double* __restrict__ partial)
{
    __shared__ double wsum[2 * kSfWaves * kSfLag];
    const int64_t cells = (int64_t)geo.n[0] * geo.n[1] * geo.n[2];
    const int blk = blockIdx.x, qi = blockIdx.y, b = blockIdx.z;
    const double* Q = q + ((int64_t)b * nq + qi) * cells;
    double* out = partial + ((int64_t)b * nq + qi) * max_h * nblk;
    const int64_t item0 = (int64_t)blk * kSfThreads * kSfSegsPerThread + threadIdx.x;

    for (int h0 = 1, ch = 0; h0 <= max_h; h0 += kSfLag, ++ch) {
        // lags past max_h are summed as well and never stored (their window stays in the line)
        double acc[kSfLag];
#pragma unroll
        for (int l = 0; l < kSfLag; ++l) acc[l] = 0.0;
#pragma unroll 1   // one segment's values in registers at a time (3 wavefronts per SIMD)
        for (int j = 0; j < kSfSegsPerThread; ++j) {
            const SfSeg sg = sf_segment(geo, item0 + (int64_t)j * kSfThreads);
            if (sg.len == 0) continue;
            // 32-bit cell indices (a field has < 2^31 cells) off the workgroup's field base
            const uint32_t base = (uint32_t)sg.base, stride = (uint32_t)sg.stride;
            double v0[kSfSeg], w[kSfWin];
#pragma unroll
            for (int r = 0; r < kSfSeg; ++r)   // positions past a ragged line's end are skipped
                v0[r] = Q[base + (uint32_t)(r < sg.len ? sg.x0 + r : sg.x0) * stride];
            uint32_t p = (uint32_t)((sg.x0 + h0) % sg.nd);
#pragma unroll
            for (int k = 0; k < kSfWin; ++k) {
                w[k] = Q[base + p * stride];
                p = (p + 1 == (uint32_t)sg.nd) ? 0u : p + 1;
            }
            sf_segment_terms(v0, w, sg.len, acc);
        }
        sf_block_store(acc, wsum, ch, h0, max_h, out, nblk, blk_off + blk);
    }
}

// Staged lines. A workgroup takes 16 lines and 16 consecutive segments of each (256 cells),
// and stages those cells plus the cells their lag windows reach (the periodic continuation,
// so no wrap remains) in LDS with loads issued all at once; every thread then takes one
// (line, segment) and reads its values and windows from LDS at fixed offsets. Lags up to
// kSfStripLags (larger max_h: sf_partial_kernel).
constexpr int kSfStripLines = 16;
constexpr int kSfStripSegs = 16;
constexpr int kSfStripSpan = kSfStripSegs * kSfSeg;                   // 256 cells per line
constexpr int kSfStripLags = 64;
constexpr int kSfStripExt = kSfStripSpan + kSfStripLags + kSfSeg;     // cells staged per line
static_assert(kSfStripLines * kSfStripSegs == kSfThreads, "one (line, segment) per thread");

// Lines along y or z: 16 lines adjacent in memory (consecutive x), stride S between a line's
// cells; tile[e][c] = cell e of line c (lanes on neighbouring lines read neighbouring slots).
// Blocks: (strip of 16 x, other coordinate, group of 16 segments); partials blk_off + blk.
__global__ void __launch_bounds__(kSfThreads)
sf_cols_kernel(const double* __restrict__ q, int32_t nx, int32_t L, int64_t S, int64_t other_stride,
               int32_t strips_x, int32_t nother, int32_t groups, int32_t nq, int32_t max_h,
               int32_t nblk, int32_t blk_off, int64_t cells, int32_t div_lo, int32_t div_hi,
               double* __restrict__ partial)
{
    __shared__ double tile[kSfStripExt * kSfStripLines];
    __shared__ double wsum[2 * kSfWaves * kSfLag];
    const int blk = blockIdx.x, qi = blockIdx.y, b = blockIdx.z;
    const int g = blk % groups, rest = blk / groups;
    const int sx = rest % strips_x, o = rest / strips_x;
    const int x0 = sx * kSfStripLines;
    const int32_t P0 = g * kSfStripSpan;                      // first cell of the group
    const int segs = (L + kSfSeg - 1) / kSfSeg;
    const int chunks = (max_h + kSfLag - 1) / kSfLag;
    const int ext = min(kSfStripExt, kSfStripSpan + chunks * kSfLag + kSfSeg);
    const double* Q = q + ((int64_t)b * nq + qi) * cells + (int64_t)o * other_stride + x0;
    const double* R = q + (int64_t)b * nq * cells + (int64_t)o * other_stride + x0;   // field 0
    const bool div = qi >= div_lo && qi < div_hi;   // uniform over the workgroup
    double* out = partial + ((int64_t)b * nq + qi) * max_h * nblk;
    {
        constexpr int NL = kSfStripExt * kSfStripLines / kSfThreads;
        double v[NL], r[NL];
        const int c = threadIdx.x & (kSfStripLines - 1);
        const bool col_ok = x0 + c < nx;
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            const int e = (threadIdx.x >> 4) + k * (kSfThreads / kSfStripLines);
            r[k] = 1.0;
            if (e < ext && col_ok) {
                int32_t p = P0 + e;
                p = (p < L) ? p : p - L;
                if (p >= L) p %= L;
                v[k] = Q[(int64_t)p * S + c];
                if (div) r[k] = R[(int64_t)p * S + c];
            }
        }
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            const int e = (threadIdx.x >> 4) + k * (kSfThreads / kSfStripLines);
            if (e < ext && col_ok) tile[e * kSfStripLines + c] = div ? v[k] * (1.0 / r[k]) : v[k];
        }
    }
    __syncthreads();
    const int c = threadIdx.x & (kSfStripLines - 1), sl = threadIdx.x >> 4;
    const int sgi = g * kSfStripSegs + sl;
    const bool ok = sgi < segs && x0 + c < nx;
    const int len = ok ? min(kSfSeg, L - sgi * kSfSeg) : 0;
    const double* T = tile + sl * kSfSeg * kSfStripLines + c;
    for (int h0 = 1, ch = 0; h0 <= max_h; h0 += kSfLag, ++ch) {
        double acc[kSfLag];
#pragma unroll
        for (int l = 0; l < kSfLag; ++l) acc[l] = 0.0;
        if (ok) {
            double v0[kSfSeg], w[kSfWin];
#pragma unroll
            for (int i = 0; i < kSfSeg; ++i) v0[i] = T[i * kSfStripLines];
            const double* W = T + h0 * kSfStripLines;
#pragma unroll
            for (int k = 0; k < kSfWin; ++k) w[k] = W[k * kSfStripLines];
            sf_segment_terms(v0, w, len, acc);
        }
        sf_block_store(acc, wsum, ch, h0, max_h, out, nblk, blk_off + blk);
    }
}

// Lines along x (rows): 16 rows, each staged with element e at e + e / 16, so that the 16
// segments of a row, which neighbouring lanes take, start 17 slots apart (different banks).
// Blocks: (group of 16 rows, group of 16 segments); partials blk_off + blk.
constexpr int kSfRowPitch = kSfStripExt + kSfStripExt / 16 + 1;

__global__ void __launch_bounds__(kSfThreads)
sf_rows_kernel(const double* __restrict__ q, int32_t L, int64_t rows, int32_t groups, int32_t nq,
               int32_t max_h, int32_t nblk, int32_t blk_off, int32_t div_lo, int32_t div_hi,
               double* __restrict__ partial)
{
    __shared__ double tile[kSfStripLines * kSfRowPitch];
    __shared__ double wsum[2 * kSfWaves * kSfLag];
    const int blk = blockIdx.x, qi = blockIdx.y, b = blockIdx.z;
    const int g = blk % groups;
    const int64_t row0 = (int64_t)(blk / groups) * kSfStripLines;
    const int32_t P0 = g * kSfStripSpan;
    const int segs = (L + kSfSeg - 1) / kSfSeg;
    const int chunks = (max_h + kSfLag - 1) / kSfLag;
    const int ext = min(kSfStripExt, kSfStripSpan + chunks * kSfLag + kSfSeg);
    const int64_t cells = rows * L;
    const double* Q = q + ((int64_t)b * nq + qi) * cells;
    const double* R0 = q + (int64_t)b * nq * cells;   // field 0 of the sample
    const bool div = qi >= div_lo && qi < div_hi;     // uniform over the workgroup
    double* out = partial + ((int64_t)b * nq + qi) * max_h * nblk;
    {
        constexpr int PER = (kSfStripExt + kSfThreads - 1) / kSfThreads;   // loads per row
        double v[kSfStripLines][PER], d[kSfStripLines][PER];
#pragma unroll
        for (int r = 0; r < kSfStripLines; ++r)
#pragma unroll
            for (int j = 0; j < PER; ++j) {
                const int e = threadIdx.x + j * kSfThreads;
                d[r][j] = 1.0;
                if (e < ext && row0 + r < rows) {
                    int32_t p = P0 + e;
                    p = (p < L) ? p : p - L;
                    if (p >= L) p %= L;
                    v[r][j] = Q[(row0 + r) * L + p];
                    if (div) d[r][j] = R0[(row0 + r) * L + p];
                }
            }
#pragma unroll
        for (int r = 0; r < kSfStripLines; ++r)
#pragma unroll
            for (int j = 0; j < PER; ++j) {
                const int e = threadIdx.x + j * kSfThreads;
                if (e < ext && row0 + r < rows)
                    tile[r * kSfRowPitch + e + (e >> 4)] = div ? v[r][j] * (1.0 / d[r][j]) : v[r][j];
            }
    }
    __syncthreads();
    const int sl = threadIdx.x & (kSfStripSegs - 1), r = threadIdx.x >> 4;
    const int sgi = g * kSfStripSegs + sl;
    const bool ok = sgi < segs && row0 + r < rows;
    const int len = ok ? min(kSfSeg, L - sgi * kSfSeg) : 0;
    const double* T = tile + r * kSfRowPitch + 17 * sl;   // element 16 sl of the row
    for (int h0 = 1, c = 0; h0 <= max_h; h0 += kSfLag, ++c) {
        double acc[kSfLag];
#pragma unroll
        for (int l = 0; l < kSfLag; ++l) acc[l] = 0.0;
        if (ok) {
            // element 16 sl + m is at T[m + (m >> 4)]; for m = h0 + k, h0 = 1 + 16 c:
            // (m >> 4) = c + ((1 + k) >> 4)
            const double* W = T + h0 + c;
            double v0[kSfSeg], w[kSfWin];
#pragma unroll
            for (int i = 0; i < kSfSeg; ++i) v0[i] = T[i];
#pragma unroll
            for (int k = 0; k < kSfWin; ++k) w[k] = W[k + ((1 + k) >> 4)];
            sf_segment_terms(v0, w, len, acc);
        }
        sf_block_store(acc, wsum, c, h0, max_h, out, nblk, blk_off + blk);
    }
}

// The staged kernels' blocks per field: rows, then y columns, then z columns (0 when max_h
// exceeds the staged lags: the general kernel takes every axis then).
struct SfStripPlan {
    bool use;
    int64_t rows_blocks, col_blocks[3];
    int32_t groups[3], strips_x;
};

static SfStripPlan sf_strip_plan(int32_t dim, const int32_t n[3], int32_t max_h)
{
    SfStripPlan p{};
    p.use = max_h <= kSfStripLags;
    if (!p.use) return p;
    for (int d = 0; d < dim; ++d) p.groups[d] = ((n[d] + kSfSeg - 1) / kSfSeg + kSfStripSegs - 1) / kSfStripSegs;
    const int64_t rows = (int64_t)n[1] * n[2];
    p.rows_blocks = (rows + kSfStripLines - 1) / kSfStripLines * p.groups[0];
    p.strips_x = (n[0] + kSfStripLines - 1) / kSfStripLines;
    if (dim >= 2) p.col_blocks[1] = (int64_t)p.strips_x * n[2] * p.groups[1];
    if (dim >= 3) p.col_blocks[2] = (int64_t)p.strips_x * n[1] * p.groups[2];
    return p;
}

// S_q(h) of every sample of the chunk: the workgroup partials of (sample, quantity, lag)
// summed in workgroup order and normalised. One thread per (sample, quantity, lag).
__global__ void sf_sum_kernel(const double* __restrict__ partial, int32_t n_out, int32_t nblk,
                              double denom, double* __restrict__ x)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_out) return;
    const double* p = partial + (int64_t)t * nblk;
    double s = p[0];
    for (int k = 1; k < nblk; ++k) s = s + p[k];
    x[t] = s / denom;
}

// Moments over samples of S_q(h), in sample order. One thread per (quantity, lag).
__global__ void sf_welford_kernel(const double* __restrict__ x, int32_t nq, int32_t max_h,
                                  int32_t batch, int64_t count0, double* __restrict__ s2mean,
                                  double* __restrict__ s2m2)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int nt = nq * max_h;
    if (t >= nt) return;
    constexpr int D = kWelfordDepth;
    double mu = s2mean[t], s2 = s2m2[t];
    double xc[D];
#pragma unroll
    for (int i = 0; i < D; ++i) xc[i] = (i < batch) ? x[(int64_t)i * nt + t] : 0.0;
    for (int32_t b0 = 0; b0 < batch; b0 += D) {
        double xn[D];
#pragma unroll
        for (int i = 0; i < D; ++i)   // the next group's loads, before this group's work
            xn[i] = (b0 + D + i < batch) ? x[(int64_t)(b0 + D + i) * nt + t] : 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const int32_t b = b0 + i;
            if (b < batch) {
                const double v = xc[i];
                const double n = (double)(count0 + b + 1);
                const double delta = v - mu;
                mu = mu + (delta / n);
                s2 = s2 + (delta * (v - mu));
            }
        }
#pragma unroll
        for (int i = 0; i < D; ++i) xc[i] = xn[i];
    }
    s2mean[t] = mu;
    s2m2[t] = s2;
}

// Multilevel Monte Carlo level differences: per fine cell, Welford over coupled samples of
// x = q(u_fine) - q(u_coarse at the parent cell) (piecewise-constant prolongation).
template <int NF, int KIND>
__global__ void __launch_bounds__(256)
welford_diff_kernel(const double* __restrict__ fine, const double* __restrict__ coarse,
                    DiffGeom geo, int32_t batch, int64_t count0, double* __restrict__ mean,
                    double* __restrict__ m2)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t cells = (int64_t)geo.nf[0] * geo.nf[1] * geo.nf[2];
    const int64_t ccells = (int64_t)geo.nc[0] * geo.nc[1] * geo.nc[2];
    if (c >= cells) return;
    const int32_t i = (int32_t)(c % geo.nf[0]);
    const int32_t j = (int32_t)((c / geo.nf[0]) % geo.nf[1]);
    const int32_t k = (int32_t)(c / ((int64_t)geo.nf[0] * geo.nf[1]));
    const int64_t pc = ((int64_t)(k / geo.r[2]) * geo.nc[1] + (j / geo.r[1])) * geo.nc[0] + (i / geo.r[0]);
    double mu[NF], s2[NF];
#pragma unroll
    for (int q = 0; q < NF; ++q) {
        mu[q] = mean[q * cells + c];
        s2[q] = m2[q * cells + c];
    }
    for (int32_t b = 0; b < batch; ++b) {
        const double* Uf = fine + (int64_t)b * NF * cells + c;
        const double* Uc = coarse + (int64_t)b * NF * ccells + pc;
        double xf[NF], xc[NF];
#pragma unroll
        for (int q = 0; q < NF; ++q) {
            xf[q] = Uf[q * cells];
            xc[q] = Uc[q * ccells];
        }
        if (KIND != 0) {
            const double irf = 1.0 / xf[0];
            const double irc = 1.0 / xc[0];
#pragma unroll
            for (int q = 1; q < ((KIND == 1) ? NF - 1 : ((KIND == 3) ? 4 : NF)); ++q) {
                xf[q] = xf[q] * irf;
                xc[q] = xc[q] * irc;
            }
        }
        const double n = (double)(count0 + b + 1);
#pragma unroll
        for (int q = 0; q < NF; ++q) {
            const double x = xf[q] - xc[q];
            const double delta = x - mu[q];
            mu[q] = mu[q] + (delta / n);
            s2[q] = s2[q] + (delta * (x - mu[q]));
        }
    }
#pragma unroll
    for (int q = 0; q < NF; ++q) {
        mean[q * cells + c] = mu[q];
        m2[q * cells + c] = s2[q];
    }
}

// Multilevel estimate on the finest grid: out = sum_l P_{l->L} mean_l, levels in order.
__global__ void mlmc_combine_kernel(const CombineArgs a, double* __restrict__ out)
{
    const int64_t cells = (int64_t)a.nfine[0] * a.nfine[1] * a.nfine[2];
    const int64_t total = cells * a.nq;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t q = t / cells, c = t % cells;
        const int32_t i = (int32_t)(c % a.nfine[0]);
        const int32_t j = (int32_t)((c / a.nfine[0]) % a.nfine[1]);
        const int32_t k = (int32_t)(c / ((int64_t)a.nfine[0] * a.nfine[1]));
        double acc = 0.0;
        for (int l = 0; l < a.nlevels; ++l) {
            const int32_t* n = a.n[l];
            const int32_t* r = a.r[l];
            const int64_t lc = (int64_t)n[0] * n[1] * n[2];
            const int64_t pc = ((int64_t)(k / r[2]) * n[1] + (j / r[1])) * n[0] + (i / r[0]);
            const double v = a.mean[l][q * lc + pc];
            acc = (l == 0) ? v : (acc + v);
        }
        out[t] = acc;
    }
}

void launch_welford_diff(int nf, int kind, const double* fine, const double* coarse,
                         const DiffGeom& geo, int32_t batch, int64_t count0, double* mean,
                         double* m2, hipStream_t s)
{
    const int64_t cells = (int64_t)geo.nf[0] * geo.nf[1] * geo.nf[2];
    const unsigned nb = (unsigned)((cells + 255) / 256);
#define FV_DIFF(NFV, K) hipLaunchKernelGGL((welford_diff_kernel<NFV, K>), dim3(nb), dim3(256), 0, s, \
                                           fine, coarse, geo, batch, count0, mean, m2)
    if (kind == 0) FV_DIFF(1, 0);
    else if (kind == 3) FV_DIFF(8, 3);
    else if (kind == 2 && nf == 2) FV_DIFF(2, 2);
    else if (kind == 2) FV_DIFF(3, 2);
    else if (nf == 3) FV_DIFF(3, 1);
    else if (nf == 4) FV_DIFF(4, 1);
    else FV_DIFF(5, 1);
#undef FV_DIFF
}

void launch_mlmc_combine(const CombineArgs& a, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(mlmc_combine_kernel, dim3(1024), dim3(256), 0, s, a, out);
}

__global__ void variance_kernel(const double* __restrict__ m2, int64_t n, double count,
                                double* __restrict__ var)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        var[i] = m2[i] / count;
}

__global__ void fill_zero_kernel(double* __restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

int sf_blocks_per_field(int32_t dim, const int32_t n[3], int32_t max_h)
{
    const SfStripPlan sp = sf_strip_plan(dim, n, max_h);
    if (sp.use) return (int)(sp.rows_blocks + sp.col_blocks[1] + sp.col_blocks[2]);
    const SfGeom g = sf_geom(dim, n, 0);
    const int64_t per = (int64_t)kSfThreads * kSfSegsPerThread;
    return (int)((g.items[dim] + per - 1) / per);
}

template <int NF, int KIND>
static void welford_launch(const double* state, int64_t cells, int32_t batch, int64_t count0,
                           double* mean, double* m2, double* qout, hipStream_t s)
{
    static_assert(NF * 64 <= 512, "one wavefront per quantity");
    const unsigned nb = (unsigned)((cells + 63) / 64);
    constexpr bool SHARE = KIND != 0;
    if (SHARE && !qout)
        hipLaunchKernelGGL((welford_kernel<NF, KIND, SHARE>), dim3(nb), dim3(64 * NF), 0, s, state,
                           cells, batch, count0, mean, m2, qout);
    else
        hipLaunchKernelGGL((welford_kernel<NF, KIND, false>), dim3(nb), dim3(64 * NF), 0, s, state,
                           cells, batch, count0, mean, m2, qout);
}

void launch_welford(int nf, int kind, const double* state, int64_t cells, int32_t batch,
                    int64_t count0, double* mean, double* m2, double* qout, hipStream_t s)
{
    if (kind == 0) welford_launch<1, 0>(state, cells, batch, count0, mean, m2, qout, s);
    else if (kind == 3) welford_launch<8, 3>(state, cells, batch, count0, mean, m2, qout, s);
    else if (kind == 2 && nf == 2) welford_launch<2, 2>(state, cells, batch, count0, mean, m2, qout, s);
    else if (kind == 2) welford_launch<3, 2>(state, cells, batch, count0, mean, m2, qout, s);
    else if (nf == 3) welford_launch<3, 1>(state, cells, batch, count0, mean, m2, qout, s);
    else if (nf == 4) welford_launch<4, 1>(state, cells, batch, count0, mean, m2, qout, s);
    else welford_launch<5, 1>(state, cells, batch, count0, mean, m2, qout, s);
}

bool sf_staged(int32_t max_h) { return max_h <= kSfStripLags; }

void launch_sf_partial(const double* q, int32_t dim, const int32_t n[3], int32_t nq, int32_t max_h,
                       int32_t batch, int kind, double* partial, hipStream_t s)
{
    const int nblk = sf_blocks_per_field(dim, n, max_h);
    const SfStripPlan sp = sf_strip_plan(dim, n, max_h);
    // quantities formed from the state as the Welford pass forms them: fields div_lo..div_hi-1
    // divided by field 0
    const int32_t div_lo = kind > 0 ? 1 : 0;
    const int32_t div_hi = kind == 1 ? nq - 1 : (kind == 3 ? 4 : (kind == 2 ? nq : 0));
    if (!sp.use) {   // sp.use == sf_staged(max_h): here q holds the quantities (kind < 0)
        hipLaunchKernelGGL(sf_partial_kernel, dim3(nblk, nq, batch), dim3(kSfThreads), 0, s, q,
                           sf_geom(dim, n, 0), nq, max_h, nblk, 0, partial);
        return;
    }
    const int64_t cells = (int64_t)n[0] * n[1] * n[2];
    hipLaunchKernelGGL(sf_rows_kernel, dim3((unsigned)sp.rows_blocks, nq, batch), dim3(kSfThreads),
                       0, s, q, n[0], (int64_t)n[1] * n[2], sp.groups[0], nq, max_h, nblk, 0,
                       div_lo, div_hi, partial);
    int64_t off = sp.rows_blocks;
    for (int d = 1; d < dim; ++d) {
        const int64_t S = (d == 1) ? n[0] : (int64_t)n[0] * n[1];
        // the other coordinate: z for y lines (stride nx ny), y for z lines (stride nx)
        const int64_t other_stride = (d == 1) ? (int64_t)n[0] * n[1] : n[0];
        const int32_t nother = (d == 1) ? n[2] : n[1];
        hipLaunchKernelGGL(sf_cols_kernel, dim3((unsigned)sp.col_blocks[d], nq, batch),
                           dim3(kSfThreads), 0, s, q, n[0], n[d], S, other_stride, sp.strips_x,
                           nother, sp.groups[d], nq, max_h, nblk, (int)off, cells, div_lo, div_hi,
                           partial);
        off += sp.col_blocks[d];
    }
}

void launch_sf_welford(const double* partial, int32_t nq, int32_t max_h, int32_t nblk,
                       int32_t batch, int64_t count0, double denom, double* x, double* s2mean,
                       double* s2m2, hipStream_t s)
{
    const int n_out = batch * nq * max_h;
    hipLaunchKernelGGL(sf_sum_kernel, dim3((n_out + 255) / 256), dim3(256), 0, s, partial, n_out,
                       nblk, denom, x);
    const int t = nq * max_h;
    hipLaunchKernelGGL(sf_welford_kernel, dim3((t + 63) / 64), dim3(64), 0, s, x, nq, max_h, batch,
                       count0, s2mean, s2m2);
}

void launch_variance(const double* m2, int64_t n, double count, double* var, hipStream_t s)
{
    hipLaunchKernelGGL(variance_kernel, dim3(1024), dim3(256), 0, s, m2, n, count, var);
}

void launch_fill_zero(double* p, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(fill_zero_kernel, dim3(1024), dim3(256), 0, s, p, n);
}

}  // namespace fvk
