// fv_stats.hip -- on-device Monte Carlo statistics (Section 2.2): per-cell mean and
// variance of the quantities over samples (Welford, samples in index order) and the
// second-order two-point structure function S_q(h) of every sample, averaged over samples.
//
// Quantities: Euler (rho, u_1..u_dim, E) with u_k = m_k * (1 / rho); scalar: the field.
#include "fv_stats.h"

namespace fvk {

// Per-cell Welford update over the samples of one batch, in sample order. One thread per
// cell keeps the running moments of every quantity in registers.
template <int NF, bool EULER>
__global__ void __launch_bounds__(256)
welford_kernel(const double* __restrict__ state, int64_t cells, int32_t batch, int64_t count0,
               double* __restrict__ mean, double* __restrict__ m2)
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
        if (EULER) {
            const double ir = 1.0 / x[0];
#pragma unroll
            for (int q = 1; q < NF - 1; ++q) x[q] = x[q] * ir;
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

// Quantity fields q[b][quantity][cells] of a chunk of samples (elementwise).
template <int NF, bool EULER>
__global__ void quantities_kernel(const double* __restrict__ state, int64_t cells, int32_t batch,
                                  double* __restrict__ q)
{
    const int64_t total = cells * batch;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = i / cells, c = i % cells;
        const double* U = state + b * NF * cells + c;
        double* Q = q + b * NF * cells + c;
        if (EULER) {
            const double ir = 1.0 / U[0];
            Q[0] = U[0];
#pragma unroll
            for (int k = 1; k < NF - 1; ++k) Q[k * cells] = U[k * cells] * ir;
            Q[(NF - 1) * cells] = U[(NF - 1) * cells];
        } else {
#pragma unroll
            for (int k = 0; k < NF; ++k) Q[k * cells] = U[k * cells];
        }
    }
}

// Partial sums over a block of cells of sum_axes (q(x + h e) - q(x))^2 for HC lags
// h = h0 .. h0 + HC - 1. Grid: (blocks per field, quantity, sample).
constexpr int kSfCellsPerBlock = 2048;
constexpr int kSfLags = 8;

__global__ void __launch_bounds__(256)
sf_partial_kernel(const double* __restrict__ q, int32_t dim, int32_t nx, int32_t ny, int32_t nz,
                  int32_t nq, int32_t max_h, int32_t nblk, double* __restrict__ partial)
{
    __shared__ double red[256];
    const int64_t cells = (int64_t)nx * ny * nz;
    const int blk = blockIdx.x, qi = blockIdx.y, b = blockIdx.z;
    const double* Q = q + ((int64_t)b * nq + qi) * cells;
    const int64_t c0 = (int64_t)blk * kSfCellsPerBlock;
    for (int h0 = 1; h0 <= max_h; h0 += kSfLags) {
        double acc[kSfLags];
#pragma unroll
        for (int l = 0; l < kSfLags; ++l) acc[l] = 0.0;
        for (int64_t c = c0 + threadIdx.x; c < c0 + kSfCellsPerBlock && c < cells; c += 256) {
            const int32_t i = (int32_t)(c % nx);
            const int32_t j = (int32_t)((c / nx) % ny);
            const int32_t k = (int32_t)(c / ((int64_t)nx * ny));
            const double v = Q[c];
            for (int d = 0; d < dim; ++d) {
#pragma unroll
                for (int l = 0; l < kSfLags; ++l) {
                    const int h = h0 + l;
                    if (h > max_h) break;
                    int64_t c2;
                    if (d == 0) {
                        int32_t i2 = i + h; if (i2 >= nx) i2 -= nx;
                        c2 = c - i + i2;
                    } else if (d == 1) {
                        int32_t j2 = j + h; if (j2 >= ny) j2 -= ny;
                        c2 = c + (int64_t)(j2 - j) * nx;
                    } else {
                        int32_t k2 = k + h; if (k2 >= nz) k2 -= nz;
                        c2 = c + (int64_t)(k2 - k) * nx * ny;
                    }
                    const double diff = Q[c2] - v;
                    acc[l] = acc[l] + (diff * diff);
                }
            }
        }
        // fixed-shape tree over the 256 threads, lag by lag
        for (int l = 0; l < kSfLags && h0 + l <= max_h; ++l) {
            red[threadIdx.x] = acc[l];
            __syncthreads();
            for (int s = 128; s > 0; s >>= 1) {
                if (threadIdx.x < s) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + s];
                __syncthreads();
            }
            if (threadIdx.x == 0)
                partial[(((int64_t)b * nq + qi) * max_h + (h0 + l - 1)) * nblk + blk] = red[0];
            __syncthreads();
        }
    }
}

// Sum the partials of each (sample, quantity, lag) in block order, normalise, and update
// the moments over samples in sample order. One thread per (quantity, lag).
__global__ void sf_welford_kernel(const double* __restrict__ partial, int32_t nq, int32_t max_h,
                                  int32_t nblk, int32_t batch, int64_t count0, double denom,
                                  double* __restrict__ s2mean, double* __restrict__ s2m2)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nq * max_h) return;
    const int qi = t / max_h, h = t % max_h;
    double mu = s2mean[t], s2 = s2m2[t];
    for (int32_t b = 0; b < batch; ++b) {
        const double* p = partial + (((int64_t)b * nq + qi) * max_h + h) * nblk;
        double s = p[0];
        for (int k = 1; k < nblk; ++k) s = s + p[k];
        const double x = s / denom;
        const double n = (double)(count0 + b + 1);
        const double delta = x - mu;
        mu = mu + (delta / n);
        s2 = s2 + (delta * (x - mu));
    }
    s2mean[t] = mu;
    s2m2[t] = s2;
}

// Multilevel Monte Carlo level differences: per fine cell, Welford over coupled samples of
// x = q(u_fine) - q(u_coarse at the parent cell) (piecewise-constant prolongation).
template <int NF, bool EULER>
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
        if (EULER) {
            const double irf = 1.0 / xf[0];
            const double irc = 1.0 / xc[0];
#pragma unroll
            for (int q = 1; q < NF - 1; ++q) {
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

void launch_welford_diff(int nf, bool euler, const double* fine, const double* coarse,
                         const DiffGeom& geo, int32_t batch, int64_t count0, double* mean,
                         double* m2, hipStream_t s)
{
    const int64_t cells = (int64_t)geo.nf[0] * geo.nf[1] * geo.nf[2];
    const unsigned nb = (unsigned)((cells + 255) / 256);
#define FV_DIFF(NFV, E) hipLaunchKernelGGL((welford_diff_kernel<NFV, E>), dim3(nb), dim3(256), 0, s, \
                                           fine, coarse, geo, batch, count0, mean, m2)
    if (!euler) FV_DIFF(1, false);
    else if (nf == 3) FV_DIFF(3, true);
    else if (nf == 4) FV_DIFF(4, true);
    else FV_DIFF(5, true);
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

int sf_blocks_per_field(int64_t cells)
{
    return (int)((cells + kSfCellsPerBlock - 1) / kSfCellsPerBlock);
}

template <int NF, bool EULER>
static void welford_launch(const double* state, int64_t cells, int32_t batch, int64_t count0,
                           double* mean, double* m2, hipStream_t s)
{
    const unsigned nb = (unsigned)((cells + 255) / 256);
    hipLaunchKernelGGL((welford_kernel<NF, EULER>), dim3(nb), dim3(256), 0, s, state, cells,
                       batch, count0, mean, m2);
}

template <int NF, bool EULER>
static void quantities_launch(const double* state, int64_t cells, int32_t batch, double* q,
                              hipStream_t s)
{
    hipLaunchKernelGGL((quantities_kernel<NF, EULER>), dim3(2048), dim3(256), 0, s, state, cells,
                       batch, q);
}

void launch_welford(int nf, bool euler, const double* state, int64_t cells, int32_t batch,
                    int64_t count0, double* mean, double* m2, hipStream_t s)
{
    if (!euler) welford_launch<1, false>(state, cells, batch, count0, mean, m2, s);
    else if (nf == 3) welford_launch<3, true>(state, cells, batch, count0, mean, m2, s);
    else if (nf == 4) welford_launch<4, true>(state, cells, batch, count0, mean, m2, s);
    else welford_launch<5, true>(state, cells, batch, count0, mean, m2, s);
}

void launch_quantities(int nf, bool euler, const double* state, int64_t cells, int32_t batch,
                       double* q, hipStream_t s)
{
    if (!euler) quantities_launch<1, false>(state, cells, batch, q, s);
    else if (nf == 3) quantities_launch<3, true>(state, cells, batch, q, s);
    else if (nf == 4) quantities_launch<4, true>(state, cells, batch, q, s);
    else quantities_launch<5, true>(state, cells, batch, q, s);
}

void launch_sf_partial(const double* q, int32_t dim, const int32_t n[3], int32_t nq, int32_t max_h,
                       int32_t batch, double* partial, hipStream_t s)
{
    const int64_t cells = (int64_t)n[0] * n[1] * n[2];
    const int nblk = sf_blocks_per_field(cells);
    hipLaunchKernelGGL(sf_partial_kernel, dim3(nblk, nq, batch), dim3(256), 0, s, q, dim, n[0], n[1],
                       n[2], nq, max_h, nblk, partial);
}

void launch_sf_welford(const double* partial, int32_t nq, int32_t max_h, int32_t nblk,
                       int32_t batch, int64_t count0, double denom, double* s2mean, double* s2m2,
                       hipStream_t s)
{
    const int t = nq * max_h;
    hipLaunchKernelGGL(sf_welford_kernel, dim3((t + 63) / 64), dim3(64), 0, s, partial, nq, max_h,
                       nblk, batch, count0, denom, s2mean, s2m2);
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
