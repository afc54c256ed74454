// fv_stats.hip -- on-device Monte Carlo statistics (Section 2.2): per-cell mean and
// variance of the quantities over samples (Welford, samples in index order) and the
// second-order two-point structure function S_q(h) of every sample, averaged over samples.
//
// Quantities: Euler (rho, u_1..u_dim, E) with u_k = m_k * (1 / rho); scalar: the field.
#include "fv_stats.h"

namespace fvk {

// Per-cell Welford update over the samples of one batch, in sample order. One thread per
// cell keeps the running moments of every quantity in registers. With qout, the quantity
// fields of the samples are also written there ([sample][quantity][cells]) for the
// structure functions, so the state is read once.
// KIND: 0 the field itself; 1 Euler (the momenta divided by rho); 2 shallow water (the
// momenta divided by h); 3 ideal MHD (the three momenta divided by rho).
template <int NF, int KIND>
__global__ void __launch_bounds__(256)
welford_kernel(const double* __restrict__ state, int64_t cells, int32_t batch, int64_t count0,
               double* __restrict__ mean, double* __restrict__ m2, double* __restrict__ qout)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cells) return;
    double mu[NF], s2[NF];
#pragma unroll
    for (int q = 0; q < NF; ++q) {
        mu[q] = mean[q * cells + c];
        s2[q] = m2[q * cells + c];
    }
    for (int32_t b = 0; b < batch; ++b) {
        const double* U = state + (int64_t)b * NF * cells + c;
        double x[NF];
#pragma unroll
        for (int q = 0; q < NF; ++q) x[q] = U[q * cells];
        if (KIND != 0) {
            const double ir = 1.0 / x[0];
#pragma unroll
            for (int q = 1; q < ((KIND == 1) ? NF - 1 : ((KIND == 3) ? 4 : NF)); ++q) x[q] = x[q] * ir;
        }
        if (qout) {
            double* Q = qout + (int64_t)b * NF * cells + c;
#pragma unroll
            for (int q = 0; q < NF; ++q) Q[q * cells] = x[q];
        }
        const double n = (double)(count0 + b + 1);
#pragma unroll
        for (int q = 0; q < NF; ++q) {
            const double delta = x[q] - mu[q];
            mu[q] = mu[q] + (delta / n);
            s2[q] = s2[q] + (delta * (x[q] - mu[q]));
        }
    }
#pragma unroll
    for (int q = 0; q < NF; ++q) {
        mean[q * cells + c] = mu[q];
        m2[q * cells + c] = s2[q];
    }
}

// Structure-function partial sums. Every line of cells along every axis is cut into segments
// of kSfSeg cells; a thread takes kSfSegsPerThread segments and, lag after lag, accumulates
// sum_cells (q(x + h e) - q(x))^2 over their cells. The values q(x + h e) of a segment form a
// window that slides by one cell per lag, so each lag costs one new load per segment instead
// of one per cell. Segments along y and z are dealt so that neighbouring lanes take
// neighbouring lines (coalesced loads); along x, neighbouring lanes take neighbouring
// segments of a row. Lags are taken kSfLagChunk at a time (register accumulators); each is
// summed over the workgroup in a fixed order (wavefront shuffles, then the four wavefronts in
// order) into one partial per workgroup. Grid: (workgroups per field, quantity, sample).
constexpr int kSfSeg = 8;
constexpr int kSfLagChunk = 16;
constexpr int kSfThreads = 256;
constexpr int kSfSegsPerThread = 4;

struct SfGeom {
    int32_t n[3];          // grid
    int32_t dim;
    int64_t lines[3];      // lines along axis d: cells / n[d]
    int64_t segs[3];       // segments per line along axis d
    int64_t items[4];      // first segment of axis d (items[dim] = total)
};

static SfGeom sf_geom(int32_t dim, const int32_t n[3])
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
        if (d < dim) acc += g.lines[d] * g.segs[d];
    }
    g.items[dim] = acc;
    for (int d = dim + 1; d < 4; ++d) g.items[d] = acc;
    return g;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = v + __shfl_xor(v, off, 64);
    return v;
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

__global__ void __launch_bounds__(kSfThreads)
sf_partial_kernel(const double* __restrict__ q, const SfGeom geo, int32_t nq, int32_t max_h,
                  int32_t nblk, double* __restrict__ partial)
{
    __shared__ double red[kSfThreads / 64][kSfLagChunk];
    const int64_t cells = (int64_t)geo.n[0] * geo.n[1] * geo.n[2];
    const int blk = blockIdx.x, qi = blockIdx.y, b = blockIdx.z;
    const double* Q = q + ((int64_t)b * nq + qi) * cells;
    const int64_t item0 = (int64_t)blk * kSfThreads * kSfSegsPerThread + threadIdx.x;

    for (int h0 = 1; h0 <= max_h; h0 += kSfLagChunk) {
        double acc[kSfLagChunk];
#pragma unroll
        for (int l = 0; l < kSfLagChunk; ++l) acc[l] = 0.0;
        for (int j = 0; j < kSfSegsPerThread; ++j) {
            const SfSeg sg = sf_segment(geo, item0 + (int64_t)j * kSfThreads);
            if (sg.len == 0) continue;
            // base values q(x0 + r) (positions past the line wrap, and are masked)
            double v0[kSfSeg], w[kSfSeg];
            int32_t p = sg.x0;
#pragma unroll
            for (int r = 0; r < kSfSeg; ++r) {
                v0[r] = Q[sg.base + p * sg.stride];
                p = (p + 1 == sg.nd) ? 0 : p + 1;
            }
            // window w[r] = q(x0 + r + h0)
            p = sg.x0 + h0;
            if (p >= sg.nd) p -= sg.nd;   // x0 < nd and h0 < nd
#pragma unroll
            for (int r = 0; r < kSfSeg; ++r) {
                w[r] = Q[sg.base + p * sg.stride];
                if (r + 1 < kSfSeg) p = (p + 1 == sg.nd) ? 0 : p + 1;
            }
#pragma unroll
            for (int l = 0; l < kSfLagChunk; ++l) {
                double a = acc[l];
#pragma unroll
                for (int r = 0; r < kSfSeg; ++r) {
                    const double df = w[r] - v0[r];
                    a = (r < sg.len) ? __builtin_fma(df, df, a) : a;
                }
                acc[l] = a;
                if (l + 1 < kSfLagChunk) {   // slide the window by one cell
#pragma unroll
                    for (int r = 0; r + 1 < kSfSeg; ++r) w[r] = w[r + 1];
                    p = (p + 1 == sg.nd) ? 0 : p + 1;
                    w[kSfSeg - 1] = (h0 + l + 1 <= max_h) ? Q[sg.base + p * sg.stride] : 0.0;
                }
            }
        }
        // workgroup sums of the chunk's lags, in a fixed order
#pragma unroll
        for (int l = 0; l < kSfLagChunk; ++l) {
            const double ws = wave_sum(acc[l]);
            if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][l] = ws;
        }
        __syncthreads();
        if (threadIdx.x < kSfLagChunk && h0 + (int)threadIdx.x <= max_h) {
            double s = red[0][threadIdx.x];
#pragma unroll
            for (int wv = 1; wv < kSfThreads / 64; ++wv) s = s + red[wv][threadIdx.x];
            partial[(((int64_t)b * nq + qi) * max_h + (h0 + threadIdx.x - 1)) * nblk + blk] = s;
        }
        __syncthreads();
    }
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
    double mu = s2mean[t], s2 = s2m2[t];
    for (int32_t b = 0; b < batch; ++b) {
        const double v = x[(int64_t)b * nt + t];
        const double n = (double)(count0 + b + 1);
        const double delta = v - mu;
        mu = mu + (delta / n);
        s2 = s2 + (delta * (v - mu));
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

int sf_blocks_per_field(int32_t dim, const int32_t n[3])
{
    const SfGeom g = sf_geom(dim, n);
    const int64_t per = (int64_t)kSfThreads * kSfSegsPerThread;
    return (int)((g.items[dim] + per - 1) / per);
}

template <int NF, int KIND>
static void welford_launch(const double* state, int64_t cells, int32_t batch, int64_t count0,
                           double* mean, double* m2, double* qout, hipStream_t s)
{
    const unsigned nb = (unsigned)((cells + 255) / 256);
    hipLaunchKernelGGL((welford_kernel<NF, KIND>), dim3(nb), dim3(256), 0, s, state, cells,
                       batch, count0, mean, m2, qout);
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

void launch_sf_partial(const double* q, int32_t dim, const int32_t n[3], int32_t nq, int32_t max_h,
                       int32_t batch, double* partial, hipStream_t s)
{
    const SfGeom g = sf_geom(dim, n);
    const int nblk = sf_blocks_per_field(dim, n);
    hipLaunchKernelGGL(sf_partial_kernel, dim3(nblk, nq, batch), dim3(kSfThreads), 0, s, q, g, nq,
                       max_h, nblk, partial);
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
