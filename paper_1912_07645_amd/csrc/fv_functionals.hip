// fv_functionals.hip -- point PDFs, joint PDFs and shell structure functions of a batch of
// samples: the statistics that Section 2.2 lists after Fjordholm, Lye and Mishra, beside the
// mean, variance and axis structure functions of fv_stats.hip.
//
// Quantities are those of the statistics: Euler (rho, u_1..u_dim, E) with u_k = m_k * (1/rho),
// shallow water (h, u_1..u_dim) with u_k = hu_k * (1/h), scalar equations the field itself.
//
// PDFs. One thread per (sample, point or pair) finds the bin of the quantity's value in FP64:
// t = ((v - lo) / (hi - lo)) * nbins, bin floor(t), the last bin also taking a value that
// rounds onto its upper edge; values below lo and values not below hi (NaN included) have a
// counter each (point PDFs), and pairs with either value outside its range share one
// (joint PDFs). Counts are added with 64-bit atomics, so they are exact in any order.
//
// Shell structure functions. S_p(h) = 1/(N |A_h|) sum_{o in A_h} sum_x |q(x + o) - q(x)|^p on
// the periodic grid, p in {1, 2}, over the cube shell A_h = {o : max_k |o_k| = h} or the ball
// shell {o : (h - 1)^2 < |o|^2 <= h^2}. One workgroup takes one tile of one quantity of one
// sample: the quantity over the tile and a periodic halo of max_h cells on every active axis
// goes into LDS, then every thread walks the shells h = 1..max_h of its cell (all threads take
// the same offsets, so the shell tests are uniform) and the workgroup sums its cells per h
// (wavefront shuffles, then the wavefronts in order). A second pass adds the tiles in order
// and divides. Sums run in another order than the definition's, so results agree with it to
// rounding (relative 1e-12 and better in the tests), not bit for bit.
#include <algorithm>
#include <vector>

#include "fv_host.h"

namespace fvk {

constexpr int kFnThreads = 256;
constexpr int kShellMaxH = 64;

// kind: 0 the field itself; 1 Euler (momenta over rho); 2 shallow water (momenta over h);
// 3 ideal MHD (the three momenta over rho).
__device__ __forceinline__ double quantity_at(const double* U, int64_t cells, int nf, int kind,
                                              int64_t c, int qi)
{
    if (kind == 0 || qi == 0 || (kind == 1 && qi == nf - 1) || (kind == 3 && qi > 3))
        return U[(int64_t)qi * cells + c];
    const double ir = 1.0 / U[c];
    return U[(int64_t)qi * cells + c] * ir;
}

// Bin 0..nbins-1; -1 below lo; nbins not below hi (NaN included).
__device__ __forceinline__ int bin_of(double v, double lo, double hi, int nbins)
{
    if (v < lo) return -1;
    if (!(v < hi)) return nbins;
    const int64_t k = (int64_t)floor(((v - lo) / (hi - lo)) * (double)nbins);
    return k < nbins ? (int)k : nbins - 1;
}

struct PdfArgs {
    const double* state;         // [batch][nf][cells]
    int64_t cells;
    int32_t nf, kind;
    int64_t batch, n;            // samples; points (or pairs)
    const int64_t* cell;         // [n] points, or [n][2] pairs
    int32_t qa, qb, nbins, joint;
    double lo_a, hi_a, lo_b, hi_b;
    unsigned long long* counts;  // [n][nbins + 2] or [n][nbins * nbins + 1]
};

__global__ void __launch_bounds__(kFnThreads) pdf_kernel(const PdfArgs a)
{
    const int64_t t = (int64_t)blockIdx.x * kFnThreads + threadIdx.x;
    if (t >= a.batch * a.n) return;
    const int64_t b = t / a.n, i = t % a.n;
    const double* U = a.state + b * a.nf * a.cells;
    if (!a.joint) {
        const int k = bin_of(quantity_at(U, a.cells, a.nf, a.kind, a.cell[i], a.qa), a.lo_a, a.hi_a, a.nbins);
        const int slot = (k < 0) ? a.nbins : (k >= a.nbins ? a.nbins + 1 : k);
        atomicAdd(&a.counts[i * (a.nbins + 2) + slot], 1ull);
    } else {
        const int ka = bin_of(quantity_at(U, a.cells, a.nf, a.kind, a.cell[2 * i], a.qa), a.lo_a, a.hi_a, a.nbins);
        const int kb = bin_of(quantity_at(U, a.cells, a.nf, a.kind, a.cell[2 * i + 1], a.qb), a.lo_b, a.hi_b, a.nbins);
        const int64_t per = (int64_t)a.nbins * a.nbins + 1;
        const bool in = ka >= 0 && ka < a.nbins && kb >= 0 && kb < a.nbins;
        atomicAdd(&a.counts[i * per + (in ? (int64_t)ka * a.nbins + kb : per - 1)], 1ull);
    }
}

// Tile of the shell kernel: 256 cells.
template <int DIM>
struct ShellTile {
    static constexpr int TX = (DIM == 1) ? 256 : (DIM == 2 ? 16 : 8);
    static constexpr int TY = (DIM == 1) ? 1 : (DIM == 2 ? 16 : 8);
    static constexpr int TZ = (DIM == 3) ? 4 : 1;
};

struct ShellArgs {
    const double* state;   // first sample of the chunk: [samples][nf][cells]
    int64_t cells;
    int32_t n[3];
    int32_t tiles[3];
    int32_t ntiles;
    int32_t nf, kind, nq, H, ball;
    double* partial;       // [sample][q][H][ntiles]
};

__device__ __forceinline__ int32_t wrap_mod(int32_t i, int32_t n)
{
    i %= n;
    return i < 0 ? i + n : i;
}

__device__ __forceinline__ bool in_ball_shell(int ox, int oy, int oz, int h)
{
    const int r2 = ox * ox + oy * oy + oz * oz;
    return (h - 1) * (h - 1) < r2 && r2 <= h * h;
}

template <int P>
__device__ __forceinline__ double shell_term(double d)
{
    return (P == 1) ? fabs(d) : (d * d);
}

template <int DIM, int P>
__global__ void __launch_bounds__(kFnThreads) shell_kernel(const ShellArgs a)
{
    using T = ShellTile<DIM>;
    constexpr int TX = T::TX, TY = T::TY, TZ = T::TZ;
    extern __shared__ double lds[];
    const int H = a.H;
    const int HY = (DIM >= 2) ? H : 0, HZ = (DIM >= 3) ? H : 0;
    const int PX = TX + 2 * H, PY = TY + 2 * HY, PZ = TZ + 2 * HZ;
    double* lq = lds;                       // quantity over tile + halo
    double* wsum = lds + PX * PY * PZ;      // [waves][H]

    const int64_t blk = blockIdx.x;
    const int32_t tile = (int32_t)(blk % a.ntiles);
    const int64_t sq = blk / a.ntiles;      // sample * nq + quantity
    const int qi = (int)(sq % a.nq);
    const int64_t b = sq / a.nq;
    const int32_t x0 = (tile % a.tiles[0]) * TX;
    const int32_t y0 = ((tile / a.tiles[0]) % a.tiles[1]) * TY;
    const int32_t z0 = (tile / (a.tiles[0] * a.tiles[1])) * TZ;
    const double* U = a.state + b * a.nf * a.cells;

    for (int e = threadIdx.x; e < PX * PY * PZ; e += kFnThreads) {
        const int px = e % PX, py = (e / PX) % PY, pz = e / (PX * PY);
        const int32_t gx = wrap_mod(x0 + px - H, a.n[0]);
        const int32_t gy = (DIM >= 2) ? wrap_mod(y0 + py - HY, a.n[1]) : 0;
        const int32_t gz = (DIM >= 3) ? wrap_mod(z0 + pz - HZ, a.n[2]) : 0;
        lq[e] = quantity_at(U, a.cells, a.nf, a.kind, ((int64_t)gz * a.n[1] + gy) * a.n[0] + gx, qi);
    }
    __syncthreads();

    const int cx = threadIdx.x % TX, cy = (threadIdx.x / TX) % TY, cz = threadIdx.x / (TX * TY);
    const bool inside = x0 + cx < a.n[0] && y0 + cy < a.n[1] && z0 + cz < a.n[2];
    const int lc = ((cz + HZ) * PY + (cy + HY)) * PX + (cx + H);
    const double q0 = lq[lc];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int h = 1; h <= H; ++h) {
        const int hy = (DIM >= 2) ? h : 0, hz = (DIM >= 3) ? h : 0;
        double acc = 0.0;
        for (int oz = -hz; oz <= hz; ++oz)
            for (int oy = -hy; oy <= hy; ++oy) {
                const double* row = lq + lc + (oz * PY + oy) * PX;
                if (a.ball) {
                    for (int ox = -h; ox <= h; ++ox)
                        if (in_ball_shell(ox, oy, oz, h)) acc = acc + shell_term<P>(row[ox] - q0);
                } else if ((DIM >= 2 && (oy == -h || oy == h)) || (DIM >= 3 && (oz == -h || oz == h))) {
                    // a row on a face of the cube (only active axes have faces)
                    for (int ox = -h; ox <= h; ++ox) acc = acc + shell_term<P>(row[ox] - q0);
                } else {
                    // an inner row of the cube: only its two ends are on the shell
                    acc = acc + shell_term<P>(row[-h] - q0);
                    acc = acc + shell_term<P>(row[h] - q0);
                }
            }
        acc = inside ? acc : 0.0;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) acc = acc + __shfl_xor(acc, off, 64);
        if (lane == 0) wsum[wave * H + (h - 1)] = acc;
    }
    __syncthreads();
    for (int h = threadIdx.x; h < H; h += kFnThreads) {
        double s = wsum[h];
        for (int w = 1; w < kFnThreads / 64; ++w) s = s + wsum[w * H + h];
        a.partial[(sq * H + h) * a.ntiles + tile] = s;
    }
}

struct ShellFinishArgs {
    const double* partial;   // [rows][ntiles], row = (sample * nq + q) * H + h - 1
    int64_t rows;
    int32_t ntiles, H;
    double cells;
    double shell[kShellMaxH];  // |A_h|
    double* out;             // [rows]
};

__global__ void __launch_bounds__(kFnThreads) shell_finish_kernel(const ShellFinishArgs a)
{
    const int64_t r = (int64_t)blockIdx.x * kFnThreads + threadIdx.x;
    if (r >= a.rows) return;
    const double* p = a.partial + r * a.ntiles;
    double s = p[0];
    for (int t = 1; t < a.ntiles; ++t) s = s + p[t];
    a.out[r] = s / (a.cells * a.shell[r % a.H]);
}

template <int DIM, int P>
static void launch_shell(const ShellArgs& a, int64_t blocks, size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL((shell_kernel<DIM, P>), dim3((unsigned)blocks), dim3(kFnThreads), lds, s, a);
}

// Number of offsets in the shell of radius h (same membership rule as the kernel).
static int64_t shell_size(int dim, int h, int ball)
{
    int64_t c = 0;
    const int hy = dim >= 2 ? h : 0, hz = dim >= 3 ? h : 0;
    for (int oz = -hz; oz <= hz; ++oz)
        for (int oy = -hy; oy <= hy; ++oy)
            for (int ox = -h; ox <= h; ++ox) {
                if (ball) {
                    const int r2 = ox * ox + oy * oy + oz * oz;
                    c += (h - 1) * (h - 1) < r2 && r2 <= h * h;
                } else {
                    c += std::max({std::abs(ox), std::abs(oy), std::abs(oz)}) == h;
                }
            }
    return c;
}

}  // namespace fvk

using namespace fvk;

static int32_t num_quantities(const fv_solver* s) { return quantity_kind(s) ? s->nf : 1; }

static fv_status pdf_common(const fv_solver* s, const double* state, int64_t batch, int32_t qa,
                            int32_t qb, int64_t n, const int64_t* cells_host, int per, double lo_a,
                            double hi_a, double lo_b, double hi_b, int32_t nbins, int64_t* counts,
                            bool joint)
{
    if (!s || !state || !counts || (n > 0 && !cells_host)) return fail(FV_EINVAL, "NULL argument");
    if (batch < 1) return fail(FV_EINVAL, "batch must be >= 1");
    if (n < 0) return fail(FV_EINVAL, "negative number of points");
    const int32_t nq = num_quantities(s);
    if (qa < 0 || qa >= nq || qb < 0 || qb >= nq) return fail(FV_EINVAL, "no such quantity");
    if (nbins < 1 || nbins > 65536) return fail(FV_EINVAL, "nbins must be in 1..65536");
    if (!(lo_a < hi_a) || !(lo_b < hi_b)) return fail(FV_EINVAL, "empty bin range (lo < hi required)");
    for (int64_t i = 0; i < n * per; ++i)
        if (cells_host[i] < 0 || cells_host[i] >= s->cells) return fail(FV_EINVAL, "cell index out of range");
    if (n == 0) return FV_OK;
    fv_solver* sm = const_cast<fv_solver*>(s);
    HIP_TRY(hipSetDevice(s->device));
    fv_status e = ensure_scratch(sm, sizeof(int64_t) * (size_t)(n * per));
    if (e) return e;
    e = stream_enter(sm);
    if (e) return e;
    HIP_TRY(hipMemcpyAsync(sm->scratch, cells_host, sizeof(int64_t) * (size_t)(n * per),
                           hipMemcpyHostToDevice, sm->stream));
    PdfArgs a{};
    a.state = state;
    a.cells = s->cells;
    a.nf = s->nf;
    a.kind = quantity_kind(s);
    a.batch = batch;
    a.n = n;
    a.cell = (const int64_t*)sm->scratch;
    a.qa = qa;
    a.qb = qb;
    a.nbins = nbins;
    a.joint = joint;
    a.lo_a = lo_a;
    a.hi_a = hi_a;
    a.lo_b = lo_b;
    a.hi_b = hi_b;
    a.counts = (unsigned long long*)counts;
    const int64_t threads = batch * n;
    hipLaunchKernelGGL(pdf_kernel, dim3((unsigned)((threads + kFnThreads - 1) / kFnThreads)),
                       dim3(kFnThreads), 0, sm->stream, a);
    HIP_TRY(hipGetLastError());
    return stream_leave(sm);
}

extern "C" fv_status fv_point_pdf(const fv_solver* solver, const double* state, int64_t batch,
                                  int32_t quantity, int64_t npoints, const int64_t* points,
                                  double lo, double hi, int32_t nbins, int64_t* counts)
{
    return pdf_common(solver, state, batch, quantity, quantity, npoints, points, 1, lo, hi, lo, hi,
                      nbins, counts, false);
}

extern "C" fv_status fv_joint_pdf(const fv_solver* solver, const double* state, int64_t batch,
                                  int32_t quantity_a, int32_t quantity_b, int64_t npairs,
                                  const int64_t* pairs, double lo_a, double hi_a, double lo_b,
                                  double hi_b, int32_t nbins, int64_t* counts)
{
    return pdf_common(solver, state, batch, quantity_a, quantity_b, npairs, pairs, 2, lo_a, hi_a,
                      lo_b, hi_b, nbins, counts, true);
}

extern "C" fv_status fv_structure_shell(const fv_solver* s, const double* state, int64_t batch,
                                        int32_t max_h, int32_t order, int32_t ball, double* out)
{
    if (!s || !state || !out) return fail(FV_EINVAL, "NULL argument");
    if (batch < 1) return fail(FV_EINVAL, "batch must be >= 1");
    if (max_h < 1 || max_h > kShellMaxH) return fail(FV_EINVAL, "max_h must be in 1..64");
    if (order != 1 && order != 2) return fail(FV_EINVAL, "order must be 1 or 2");
    if (ball != 0 && ball != 1) return fail(FV_EINVAL, "ball must be 0 or 1");
    const int dim = s->grid.dim;
    for (int k = 0; k < dim; ++k) {
        if (s->grid.bc[k] != FV_BC_PERIODIC) return fail(FV_ENOTSUP, "shell structure functions need periodic axes");
        if (max_h >= s->grid.n[k]) return fail(FV_ENOTSUP, "max_h must be below the cells of every axis");
    }
    const int T[3] = {dim == 1 ? 256 : (dim == 2 ? 16 : 8), dim == 1 ? 1 : (dim == 2 ? 16 : 8), dim == 3 ? 4 : 1};
    const int64_t P[3] = {T[0] + 2 * max_h, dim >= 2 ? T[1] + 2 * max_h : 1, dim >= 3 ? T[2] + 2 * max_h : 1};
    const size_t lds = sizeof(double) * (size_t)(P[0] * P[1] * P[2] + (kFnThreads / 64) * max_h);
    if (lds > 65536) return fail(FV_ENOTSUP, "max_h too large for this dimension (tile and halo exceed 64 KB of LDS)");
    ShellArgs a{};
    a.cells = s->cells;
    a.ntiles = 1;
    for (int k = 0; k < 3; ++k) {
        a.n[k] = (int32_t)s->grid.n[k];
        a.tiles[k] = (int32_t)((s->grid.n[k] + T[k] - 1) / T[k]);
        a.ntiles *= a.tiles[k];
    }
    a.nf = s->nf;
    a.kind = quantity_kind(s);
    a.nq = num_quantities(s);
    a.H = max_h;
    a.ball = ball;
    ShellFinishArgs f{};
    f.ntiles = a.ntiles;
    f.H = max_h;
    f.cells = (double)s->cells;
    for (int h = 1; h <= max_h; ++h) f.shell[h - 1] = (double)shell_size(dim, h, ball);
    // samples per pass: partial sums of at most 2^22 doubles (32 MiB)
    const int64_t per_sample = (int64_t)a.nq * max_h * a.ntiles;
    const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(batch, (int64_t(1) << 22) / per_sample));
    fv_solver* sm = const_cast<fv_solver*>(s);
    HIP_TRY(hipSetDevice(s->device));
    fv_status e = ensure_scratch(sm, sizeof(double) * (size_t)(chunk * per_sample));
    if (e) return e;
    e = stream_enter(sm);
    if (e) return e;
    a.partial = (double*)sm->scratch;
    f.partial = a.partial;
    for (int64_t b0 = 0; b0 < batch; b0 += chunk) {
        const int64_t nb = std::min<int64_t>(chunk, batch - b0);
        a.state = state + b0 * s->nf * s->cells;
        const int64_t blocks = nb * a.nq * a.ntiles;
        switch (dim * 10 + order) {
            case 11: launch_shell<1, 1>(a, blocks, lds, sm->stream); break;
            case 12: launch_shell<1, 2>(a, blocks, lds, sm->stream); break;
            case 21: launch_shell<2, 1>(a, blocks, lds, sm->stream); break;
            case 22: launch_shell<2, 2>(a, blocks, lds, sm->stream); break;
            case 31: launch_shell<3, 1>(a, blocks, lds, sm->stream); break;
            default: launch_shell<3, 2>(a, blocks, lds, sm->stream); break;
        }
        f.rows = nb * a.nq * max_h;
        f.out = out + b0 * a.nq * max_h;
        hipLaunchKernelGGL(shell_finish_kernel, dim3((unsigned)((f.rows + kFnThreads - 1) / kFnThreads)),
                           dim3(kFnThreads), 0, sm->stream, f);
        HIP_TRY(hipGetLastError());
    }
    return stream_leave(sm);
}
