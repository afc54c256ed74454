// fv_small.hip -- the whole time loop of a small 1D problem in one workgroup per sample.
//
// A 1D grid of up to a few thousand cells is latency-bound on the tiled path: each step is a
// handful of tiny launches (stages and the step decision) of a few microseconds each. Here one
// workgroup of 1024 threads (512 for the heaviest faces) keeps its sample's state in LDS (with the ghost layers) and U^n in
// registers, and runs every step on the chip: the step decision, the stages (faces into LDS,
// divergence and Runge--Kutta combination, ghost refresh) and the wave-speed reduction, until
// the sample stops or has taken `chunk` steps in this launch (the host launches again while
// samples run, so no launch runs unboundedly). The arithmetic of each face, update and speed
// is the tiled kernels' own
// (the same device functions, in the same order), and the decision repeats the control
// kernel's rules, so the results equal the tiled path's bit for bit.
#include "fv_small.h"
#include "fv_stage.h"

namespace fvk {

// Threads per workgroup: 1024, or 512 where a face needs more registers than 1024 threads
// leave (128 each): ideal MHD's eight fields and the Euler Godunov flux's Newton iteration.
template <int EQ, int FLUX>
constexpr int small_threads() { return (EQ == EQ_MHD || (EQ == EQ_EULER && FLUX == FLUX_GODUNOV)) ? 512 : 1024; }

// Cells per thread: 4 for a scalar equation, 2 for small systems (3 with 512 threads), 1 for
// MHD (LDS caps its grids below the thread count).
template <int EQ, int FLUX>
constexpr int small_cpt()
{
    constexpr int NF = NumFields<1, EQ>::value;
    return NF >= 5 ? 1 : (NF >= 2 ? (small_threads<EQ, FLUX>() == 512 ? 3 : 2) : 4);
}

template <int EQ, int RECON, int FLUX>
__global__ void __launch_bounds__((small_threads<EQ, FLUX>())) small1d_kernel(const SmallArgs a)
{
    constexpr int NF = NumFields<1, EQ>::value;
    constexpr int G = Ghost<RECON>::value;
    constexpr int NT = small_threads<EQ, FLUX>();
    constexpr int kSmallMaxCpt = small_cpt<EQ, FLUX>();
    extern __shared__ double lds[];
    const int n = a.n;
    const int PX = n + 2 * G;
    double* su = lds;                    // [NF][PX] state with ghost layers
    double* sf = lds + NF * PX;          // [NF][n + 1] face fluxes
    __shared__ double red[NT / 64];
    __shared__ int redbad;

    const int64_t b = blockIdx.x;
    if (!a.first && !a.running[b]) return;   // uniform across the workgroup
    double* U = a.state + b * NF * (int64_t)n;
    const Phys& ph = a.ph;

    double un[kSmallMaxCpt][NF];   // U^n of the thread's cells
#pragma unroll
    for (int k = 0; k < kSmallMaxCpt; ++k) {
        const int c = threadIdx.x + k * NT;
        if (c < n) {
#pragma unroll
            for (int q = 0; q < NF; ++q) {
                un[k][q] = U[q * n + c];
                su[q * PX + G + c] = un[k][q];
            }
        }
    }
    __syncthreads();
    auto fill_ghosts = [&]() {
        for (int e = threadIdx.x; e < NF * 2 * G; e += NT) {
            const int q = e / (2 * G), j = e % (2 * G);
            const int i = (j < G) ? (j - G) : (n + j - G);     // -G..-1, n..n+G-1
            su[q * PX + G + i] = su[q * PX + G + wrap_index(i, n, a.bc)];
        }
    };
    fill_ghosts();

    // wave speed and physicality of the thread's cells of a state held in registers
    auto reduce_speed = [&](double (&v)[kSmallMaxCpt][NF], double& M, bool& bad) {
        double m = 0.0;
        bool bd = false;
#pragma unroll
        for (int k = 0; k < kSmallMaxCpt; ++k) {
            const int c = threadIdx.x + k * NT;
            if (c < n) {
                bool bk;
                const double s = cell_speed<1, EQ>(v[k], ph, bk);
                m = vmax(m, s);
                bd = bd || bk;
            }
        }
        if (threadIdx.x == 0) redbad = 0;
        __syncthreads();
        m = wave_max(m);
        if (bd) atomicOr(&redbad, 1);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
        __syncthreads();
        double r = red[0];
#pragma unroll
        for (int w = 1; w < NT / 64; ++w) r = vmax(r, red[w]);
        M = r;
        bad = redbad != 0;
        __syncthreads();   // red and redbad are reused by the next reduction
    };

    double M;
    bool bad;
    reduce_speed(un, M, bad);

    double t = a.fixed ? 0.0 : a.t[b];
    int64_t steps = a.first ? 0 : a.steps[b];
    int32_t err = ST_OK;
    bool running = true;
    for (int64_t it = 0; it < a.chunk; ++it) {
        // the step decision (every thread takes it alike from uniform values)
        double dt;
        running = false;
        if (bad) {
            err = ST_ENONPHYS;
            break;
        }
        if (a.fixed) {
            if (steps >= a.max_steps) break;
            if (a.fixed_dt * M > a.cfl_bound) {
                err = ST_ECFL;
                break;
            }
            dt = a.fixed_dt;
        } else {
            if (!(t < a.t_end)) break;
            if (steps >= a.max_steps) {
                if (a.limit_is_error) err = ST_EMAXSTEPS;
                break;
            }
            dt = (M == 0.0) ? (a.t_end - t) : (a.cfl / M);
            bool last = false;
            if (t + dt >= a.t_end) {
                dt = a.t_end - t;
                last = true;
            }
            t = last ? a.t_end : (t + dt);
        }
        steps = steps + 1;
        running = true;

        double out[kSmallMaxCpt][NF];
        for (int st = 0; st < a.nst; ++st) {
            // faces f = 0..n between cells f - 1 and f
            for (int f = threadIdx.x; f <= n; f += NT) {
                double UL[NF], UR[NF], F[NF];
#pragma unroll
                for (int q = 0; q < NF; ++q) {
                    const double* s = su + q * PX + G + f;
                    if (RECON == REC_FIRST) {
                        reconstruct<RECON>(0.0, s[-1], s[0], 0.0, UL[q], UR[q]);
                    } else {
                        reconstruct<RECON>(s[-2], s[-1], s[0], s[1], UL[q], UR[q]);
                    }
                }
                numflux<1, EQ, FLUX>(UL, UR, 0, F, ph);
#pragma unroll
                for (int q = 0; q < NF; ++q) sf[q * (n + 1) + f] = F[q];
            }
            __syncthreads();
            // divergence and stage combination of the thread's cells
            const double beta = a.beta[st];
            const bool use_un = st > 0;
#pragma unroll
            for (int k = 0; k < kSmallMaxCpt; ++k) {
                const int c = threadIdx.x + k * NT;
                if (c < n) {
#pragma unroll
                    for (int q = 0; q < NF; ++q) {
                        const double acc = (sf[q * (n + 1) + c + 1] - sf[q * (n + 1) + c]) * ph.inv_dx[0];
                        const double rhs = -acc;
                        const double up = su[q * PX + G + c];
                        const double u0 = use_un ? un[k][q] : up;
                        out[k][q] = u0 + (beta * ((up - u0) + (dt * rhs)));
                        // in this phase a thread reads only its own cells' state, so the new
                        // value can replace it at once
                        su[q * PX + G + c] = out[k][q];
                    }
                }
            }
            __syncthreads();
            fill_ghosts();
            __syncthreads();
        }
#pragma unroll
        for (int k = 0; k < kSmallMaxCpt; ++k)
#pragma unroll
            for (int q = 0; q < NF; ++q) un[k][q] = out[k][q];
        reduce_speed(un, M, bad);
    }

#pragma unroll
    for (int k = 0; k < kSmallMaxCpt; ++k) {
        const int c = threadIdx.x + k * NT;
        if (c < n) {
#pragma unroll
            for (int q = 0; q < NF; ++q) U[q * n + c] = un[k][q];
        }
    }
    if (threadIdx.x == 0) {
        if (!a.fixed) a.t[b] = t;
        a.steps[b] = steps;
        a.err[b] = err;
        a.running[b] = running ? 1 : 0;
        if (running) atomicAdd(a.n_running, 1);
    }
}

template <int EQ, int RECON, int FLUX>
static void launch_small(const SmallArgs& a, hipStream_t s)
{
    constexpr int NF = NumFields<1, EQ>::value;
    constexpr int G = Ghost<RECON>::value;
    const size_t lds = sizeof(double) * (size_t)NF * ((a.n + 2 * G) + (a.n + 1));
    hipLaunchKernelGGL((small1d_kernel<EQ, RECON, FLUX>), dim3((unsigned)a.batch),
                       dim3(small_threads<EQ, FLUX>()), lds, s, a);
}

template <int EQ, int RECON, int FLUX>
constexpr SmallKernel make_small()
{
    constexpr int NF = NumFields<1, EQ>::value;
    constexpr int G = Ghost<RECON>::value;
    // LDS of the state with ghosts and the faces within 60 KiB, and the cells per thread
    constexpr int by_lds = (60 * 1024 / (8 * NF) - 2 * G - 1) / 2;
    constexpr int cap = small_threads<EQ, FLUX>() * small_cpt<EQ, FLUX>();
    return SmallKernel{EQ, RECON, FLUX, &launch_small<EQ, RECON, FLUX>, by_lds < cap ? by_lds : cap};
}

#define SMALL4(E, F) make_small<E, REC_FIRST, F>(), make_small<E, REC_MUSCL, F>(), \
                     make_small<E, REC_WENO3, F>(), make_small<E, REC_ENO2, F>()
static const SmallKernel kSmall[] = {
    SMALL4(EQ_EULER, FLUX_RUSANOV), SMALL4(EQ_EULER, FLUX_HLL), SMALL4(EQ_EULER, FLUX_HLLC),
    SMALL4(EQ_EULER, FLUX_ROE), SMALL4(EQ_EULER, FLUX_GODUNOV), SMALL4(EQ_EULER, FLUX_EC),
    SMALL4(EQ_BURGERS, FLUX_RUSANOV), SMALL4(EQ_BURGERS, FLUX_HLL), SMALL4(EQ_BURGERS, FLUX_ROE),
    SMALL4(EQ_BURGERS, FLUX_GODUNOV), SMALL4(EQ_BURGERS, FLUX_EC),
    SMALL4(EQ_ADVECTION, FLUX_RUSANOV), SMALL4(EQ_ADVECTION, FLUX_HLL), SMALL4(EQ_ADVECTION, FLUX_ROE),
    SMALL4(EQ_ADVECTION, FLUX_GODUNOV),
    SMALL4(EQ_SWE, FLUX_RUSANOV), SMALL4(EQ_SWE, FLUX_HLL), SMALL4(EQ_SWE, FLUX_ROE),
    SMALL4(EQ_MHD, FLUX_RUSANOV), SMALL4(EQ_MHD, FLUX_HLL),
};
#undef SMALL4

const SmallKernel* find_small_kernel(int eq, int recon, int flux)
{
    for (const SmallKernel& k : kSmall)
        if (k.eq == eq && k.recon == recon && k.flux == flux) return &k;
    return nullptr;
}

}  // namespace fvk
