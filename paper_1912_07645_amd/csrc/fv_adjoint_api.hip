// fv_adjoint_api.hip -- host side of the discrete adjoint: fixed-dt forward run with
// checkpoints, reverse sweep with per-segment recomputation, the kinetic-energy quantity of
// interest and the line-wise contraction with the initial-data derivative.
//
// Checkpointing, two policies.
// - Segments: the state is stored every `every` steps (every = ceil(sqrt(nsteps)) gives the
//   classical sqrt(N) scheme). The reverse sweep takes the segments last to first; each is
//   recomputed forward from its checkpoint with all Runge--Kutta stage states stored, then
//   reversed stage by stage. Memory: ceil(N / every) + every * stages + 4 states per batch.
// - Binomial (Griewank's revolve schedule): only the initial state is kept from the forward
//   run, plus `snapshots` free checkpoint slots. Reversing l steps with s free slots from a
//   stored state at n0 advances to n0 + m, stores that state in a slot, reverses the last
//   l - m steps with s - 1 slots, then the first m with s. With the split m chosen as below,
//   the reverse sweep runs p(l, s + 1) + l forward steps, p the binomial minimum
//   t l - C(s + 1 + t, t - 1) with C(s + t, t - 1) < l <= C(s + 1 + t, t) (Griewank 1992);
//   memory snapshots + stages + 5 states per batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <new>
#include <vector>

#include "fv_adjoint.h"
#include "fv_host.h"

using namespace fvk;

struct fv_adjoint {
    fv_solver* s = nullptr;
    const AdjKernel* ak = nullptr;
    int64_t batch = 0, nsteps = 0, every = 0, nseg = 0;
    bool binomial = false;
    int64_t snapshots = 0;         // binomial: free checkpoint slots besides the initial state
    double* snap = nullptr;        // binomial: snapshots states
    int64_t recomputed = 0;        // forward steps run by the last reverse sweep
    double dt = 0.0, cfl_bound = 0.0;
    int nst = 0;
    size_t state_doubles = 0;      // doubles per batch state
    double* ckpt = nullptr;        // nseg states
    double* seg = nullptr;         // every * nst + 1 states
    double* lam[3] = {nullptr, nullptr, nullptr};
    double* dt_arr = nullptr;      // [batch]
    int32_t* active = nullptr;     // [batch], all 1
    unsigned long long* mbits = nullptr;
    int32_t* bad = nullptr;
    bool forward_done = false;
    unsigned long long* sig = nullptr;   // caller's branch-signature sums (diagnostic)
    unsigned long long rev_launch = 0;   // reverse stage launches of the current sweep
};

static __global__ void adj_init_kernel(double* dt_arr, int32_t* active, unsigned long long* mbits,
                                       int32_t* bad, int64_t batch, double dt)
{
    const int64_t pitch = speed_pitch(batch);
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < batch;
         b += (int64_t)gridDim.x * blockDim.x) {
        dt_arr[b] = dt;
        active[b] = 1;
        for (int s = 0; s < kSpeedSlots; ++s) mbits[s * pitch + b] = 0ull;
        bad[b] = 0;
    }
}

static Group stage_group(const fv_adjoint* a, const double* src, const double* un, double* dst)
{
    const fv_solver* s = a->s;
    Group g{};
    g.src = src;
    g.un = un;
    g.dst = dst;
    g.dt = a->dt_arr;
    g.active = a->active;
    g.mbits = a->mbits;
    g.bad = a->bad;
    g.cells = s->cells;
    const int32_t tb[3] = {s->kern->bx, s->kern->by, s->kern->bz};
    g.ntiles = 1;
    for (int k = 0; k < 3; ++k) {
        g.n[k] = (int32_t)s->grid.n[k];
        g.tiles[k] = (int32_t)((s->grid.n[k] + tb[k] - 1) / tb[k]);
        g.ntiles *= g.tiles[k];
    }
    g.batch = (int32_t)a->batch;
    g.block0 = 0;
    g.ph = s->ph;
    return g;
}

// One forward step from `un` with stage outputs to dst[0..nst-1] (dst[nst-1] = next state).
static void forward_step(const fv_adjoint* a, const double* un, double* const* dst)
{
    const fv_solver* s = a->s;
    const double* src = un;
    for (int st = 0; st < a->nst; ++st) {
        StageArgs sa{};
        sa.ngroups = 1;
        sa.g[0] = stage_group(a, src, un, dst[st]);
        for (int k = 0; k < 3; ++k) sa.bc[k] = s->grid.bc[k];
        sa.beta = stage_beta(s->integ, st);
        sa.use_un = st > 0;
        sa.last = (st == a->nst - 1);
        sa.nblocks = (int64_t)sa.g[0].ntiles * a->batch;
        s->kern->stage(sa, s->stream);
        src = dst[st];
    }
}

static fv_status adjoint_create(fv_solver* s, int64_t batch, int64_t nsteps, double dt,
                                int64_t every, int64_t snapshots, bool binomial, double cfl_bound,
                                fv_adjoint** out)
{
    if (!s || !out) return fail(FV_EINVAL, "NULL argument");
    *out = nullptr;
    if (batch < 1 || nsteps < 1) return fail(FV_EINVAL, "batch and nsteps must be >= 1");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(FV_EINVAL, "dt must be > 0");
    if (!(cfl_bound > 0.0)) return fail(FV_EINVAL, "cfl_bound must be > 0");
    const AdjKernel* ak = find_adjoint_kernel(s->grid.dim, s->eq.kind, s->recon, s->flux);
    if (!ak)
        return fail(FV_ENOTSUP, "the adjoint covers the Euler equations in 1D/2D with the Rusanov "
                                "flux and first-order or MUSCL-minmod reconstruction");
    for (int k = 0; k < s->grid.dim; ++k)
        if (s->grid.bc[k] != FV_BC_PERIODIC)
            return fail(FV_ENOTSUP, "the adjoint covers periodic grids only (a transmissive "
                                    "boundary face has terms the reverse stage does not add)");
    if (binomial) {
        if (snapshots < 0) return fail(FV_EINVAL, "snapshots must be >= 0");
        snapshots = std::min(snapshots, nsteps);
        every = nsteps;   // the forward run keeps the initial state only
    } else {
        if (every <= 0) every = (int64_t)std::ceil(std::sqrt((double)nsteps));
        every = std::min(every, nsteps);
    }
    const int64_t tiles = [&] {
        int64_t n = 1;
        const int32_t tb[3] = {ak->bx, ak->by, ak->bz};
        for (int k = 0; k < 3; ++k) n *= (s->grid.n[k] + tb[k] - 1) / tb[k];
        return n;
    }();
    if (tiles * batch > 0x7fffffffLL) return fail(FV_EINVAL, "launch too large");
    fv_adjoint* a = new (std::nothrow) fv_adjoint();
    if (!a) return fail(FV_ENOMEM, "host allocation failed");
    a->s = s;
    a->ak = ak;
    a->batch = batch;
    a->nsteps = nsteps;
    a->every = every;
    a->nseg = (nsteps + every - 1) / every;
    a->binomial = binomial;
    a->snapshots = snapshots;
    a->dt = dt;
    a->cfl_bound = cfl_bound;
    a->nst = n_stages(s->integ);
    a->state_doubles = (size_t)batch * s->nf * s->cells;
    const size_t sb = sizeof(double) * a->state_doubles;
    // segment states: every step's stages (segments), or one step's stages plus two work
    // states (binomial)
    const int64_t nseg_states = binomial ? a->nst + 2 : every * a->nst + 1;
    bool ok = hipSetDevice(s->device) == hipSuccess &&
              hipMalloc((void**)&a->ckpt, sb * a->nseg) == hipSuccess &&
              hipMalloc((void**)&a->seg, sb * nseg_states) == hipSuccess &&
              (!binomial || snapshots == 0 ||
               hipMalloc((void**)&a->snap, sb * snapshots) == hipSuccess) &&
              hipMalloc((void**)&a->lam[0], sb) == hipSuccess &&
              hipMalloc((void**)&a->lam[1], sb) == hipSuccess &&
              hipMalloc((void**)&a->lam[2], sb) == hipSuccess &&
              hipMalloc((void**)&a->dt_arr, sizeof(double) * batch) == hipSuccess &&
              hipMalloc((void**)&a->active, sizeof(int32_t) * batch) == hipSuccess &&
              hipMalloc((void**)&a->mbits, sizeof(unsigned long long) * kSpeedSlots * speed_pitch(batch)) == hipSuccess &&
              hipMalloc((void**)&a->bad, sizeof(int32_t) * batch) == hipSuccess;
    if (!ok) {
        fv_adjoint_destroy(a);
        return fail(FV_ENOMEM, "adjoint allocation failed");
    }
    *out = a;
    return FV_OK;
}

extern "C" fv_status fv_adjoint_create(fv_solver* s, int64_t batch, int64_t nsteps, double dt,
                                       int64_t every, double cfl_bound, fv_adjoint** out)
{
    return adjoint_create(s, batch, nsteps, dt, every, 0, false, cfl_bound, out);
}

extern "C" fv_status fv_adjoint_create_binomial(fv_solver* s, int64_t batch, int64_t nsteps,
                                                double dt, int64_t snapshots, double cfl_bound,
                                                fv_adjoint** out)
{
    return adjoint_create(s, batch, nsteps, dt, 0, snapshots, true, cfl_bound, out);
}

extern "C" fv_status fv_adjoint_recomputed_steps(const fv_adjoint* a, int64_t* steps)
{
    if (!a || !steps) return fail(FV_EINVAL, "NULL argument");
    *steps = a->recomputed;
    return FV_OK;
}

extern "C" fv_status fv_adjoint_set_signature(fv_adjoint* a, uint64_t* sig)
{
    if (!a) return fail(FV_EINVAL, "adjoint is NULL");
    a->sig = (unsigned long long*)sig;
    return FV_OK;
}

extern "C" fv_status fv_adjoint_destroy(fv_adjoint* a)
{
    if (!a) return FV_OK;
    if (a->s && a->s->stream) hipStreamSynchronize(a->s->stream);
    hipFree(a->ckpt);
    hipFree(a->seg);
    hipFree(a->snap);
    for (double* l : a->lam) hipFree(l);
    hipFree(a->dt_arr);
    hipFree(a->active);
    hipFree(a->mbits);
    hipFree(a->bad);
    delete a;
    return FV_OK;
}

extern "C" fv_status fv_adjoint_forward(fv_adjoint* a, const double* state0, double* stateT)
{
    if (!a || !state0 || !stateT) return fail(FV_EINVAL, "NULL argument");
    fv_solver* s = a->s;
    HIP_TRY(hipSetDevice(s->device));
    fv_status e = stream_enter(s);
    if (e) return e;
    hipStream_t st = s->stream;
    const size_t sb = sizeof(double) * a->state_doubles;
    hipLaunchKernelGGL(adj_init_kernel, dim3(64), dim3(256), 0, st, a->dt_arr, a->active, a->mbits,
                       a->bad, a->batch, a->dt);
    {   // wave speed and physicality of the initial state
        SpeedArgs sp{};
        sp.ngroups = 1;
        sp.g[0] = stage_group(a, state0, state0, nullptr);
        sp.nblocks = ((s->cells + s->kern->cells_per_block - 1) / s->kern->cells_per_block) * a->batch;
        s->kern->speed(sp, st);
    }
    // rolling buffers: seg[0] holds the current state, seg[1..] the stage states
    double* cur = a->seg;
    HIP_TRY(hipMemcpyAsync(cur, state0, sb, hipMemcpyDeviceToDevice, st));
    std::vector<double*> dst(a->nst);
    for (int k = 0; k < a->nst - 1; ++k) dst[k] = a->seg + (size_t)(k + 1) * a->state_doubles;
    double* other = a->seg + (size_t)a->nst * a->state_doubles;  // forward Euler needs a second buffer
    for (int64_t n = 0; n < a->nsteps; ++n) {
        if (n % a->every == 0)
            HIP_TRY(hipMemcpyAsync(a->ckpt + (size_t)(n / a->every) * a->state_doubles, cur, sb,
                                   hipMemcpyDeviceToDevice, st));
        if (a->nst == 1) {
            dst[0] = other;
            forward_step(a, cur, dst.data());
            std::swap(cur, other);
        } else {
            dst[a->nst - 1] = cur;   // last stage writes U^{n+1} in place over U^n
            forward_step(a, cur, dst.data());
        }
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(stateT, cur, sb, hipMemcpyDeviceToDevice, st));
    // trajectory checks: max wave speed over all states, non-physical values
    const int64_t pitch = speed_pitch(a->batch);
    std::vector<unsigned long long> mb((size_t)(kSpeedSlots * pitch));
    std::vector<int32_t> bd((size_t)a->batch);
    HIP_TRY(hipMemcpyAsync(mb.data(), a->mbits, sizeof(unsigned long long) * mb.size(), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(bd.data(), a->bad, sizeof(int32_t) * a->batch, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    a->forward_done = true;
    e = stream_leave(s);
    if (e) return e;
    for (int64_t b = 0; b < a->batch; ++b) {
        unsigned long long mx = 0ull;   // bit patterns of non-negative doubles order like them
        for (int s2 = 0; s2 < kSpeedSlots; ++s2) mx = std::max(mx, mb[(size_t)(s2 * pitch + b)]);
        double M;
        std::memcpy(&M, &mx, sizeof(double));
        if (bd[(size_t)b]) return fail(FV_ENONPHYS, "sample " + std::to_string(b) + " became non-physical");
        if (a->dt * M > a->cfl_bound)
            return fail(FV_ECFL, "sample " + std::to_string(b) + ": dt * max speed exceeded the bound");
    }
    return FV_OK;
}

static fv_status reverse_stage(fv_adjoint* a, const double* U, const double* lam, double* prev,
                               double* acc, int mode, double beta)
{
    const fv_solver* s = a->s;
    AdjArgs g{};
    g.U = U;
    g.lam = lam;
    g.prev = prev;
    g.acc = acc;
    g.cells = s->cells;
    g.ntiles = 1;
    const int32_t tb[3] = {a->ak->bx, a->ak->by, a->ak->bz};
    for (int k = 0; k < 3; ++k) {
        g.n[k] = (int32_t)s->grid.n[k];
        g.tiles[k] = (int32_t)((s->grid.n[k] + tb[k] - 1) / tb[k]);
        g.ntiles *= g.tiles[k];
        g.bc[k] = s->grid.bc[k];
    }
    g.batch = (int32_t)a->batch;
    g.mode = mode;
    g.beta = beta;
    g.dt = a->dt;
    g.nblocks = (int64_t)g.ntiles * a->batch;
    g.ph = s->ph;
    g.sig = a->sig;
    g.salt = 0x2545F4914F6CDD1Dull * (++a->rev_launch);
    a->ak->launch(g, s->stream);
    return FV_OK;
}

// Reverse one step: stages[k] holds the state stage k of the step starts from (stages[0] =
// U^n). lam[*cur] holds dQ/dU^{n+1} on entry and dQ/dU^n on return.
static void reverse_step(fv_adjoint* a, const double* const* stages, int& cur)
{
    const fv_solver* s = a->s;
    const int S = a->nst;
    int in = cur, p = (cur + 1) % 3, acc = (cur + 2) % 3;
    if (S == 1) {
        reverse_stage(a, stages[0], a->lam[in], a->lam[p], a->lam[acc], 0, 1.0);
        cur = p;
        return;
    }
    for (int stg = S - 1; stg >= 0; --stg) {
        const double beta = stage_beta(s->integ, stg);
        const int mode = (stg == S - 1) ? 0 : (stg == 0 ? 2 : 1);
        reverse_stage(a, stages[stg], a->lam[in], a->lam[p], a->lam[acc], mode, beta);
        std::swap(in, p);   // this stage's output is the next stage's input
    }
    cur = in;
}

// Binomial coefficient C(s + t, t) for s, t >= 0, saturated at 2^62 (far above any step
// count); 0 for t < 0.
static int64_t binom_st(int64_t s, int64_t t)
{
    if (t < 0) return 0;
    const int64_t k = std::min(s, t), n = s + t;
    const unsigned __int128 cap = (unsigned __int128)1 << 62;
    unsigned __int128 r = 1;
    for (int64_t i = 1; i <= k; ++i) {
        r = (r * (unsigned __int128)(n - k + i)) / (unsigned __int128)i;   // C(n - k + i, i)
        if (r >= cap) return (int64_t)cap;
    }
    return (int64_t)r;
}

// The split of the binomial schedule: reversing l >= 2 steps with s >= 1 free slots (s + 1
// states counting the stored one), store the state after m steps, where t is the smallest
// integer with C(s + 1 + t, t) >= l and m = min(C(s + t, t - 1), l - C(s + t - 1, t - 1)),
// the largest split that keeps the binomial minimum.
static int64_t binomial_split(int64_t l, int64_t s)
{
    const int64_t snaps = s + 1;
    int64_t t = 0;
    while (binom_st(snaps, t) < l) ++t;
    int64_t m = std::min(binom_st(snaps, t - 1), l - binom_st(snaps - 1, t - 1));
    return std::max<int64_t>(1, std::min(m, l - 1));
}

// Advance k steps from the state `from` into a work buffer; returns the buffer holding the
// result (`from` itself when k = 0).
static const double* advance(fv_adjoint* a, const double* from, int64_t k)
{
    if (k == 0) return from;
    const size_t sd = a->state_doubles;
    const size_t sb = sizeof(double) * sd;
    hipStream_t st = a->s->stream;
    double* w0 = a->seg + (size_t)(a->nst + 0) * sd;   // two work states after the stage slots
    double* w1 = a->seg + (size_t)(a->nst + 1) * sd;
    hipMemcpyAsync(w0, from, sb, hipMemcpyDeviceToDevice, st);
    std::vector<double*> dst(a->nst);
    for (int j = 0; j < a->nst - 1; ++j) dst[j] = a->seg + (size_t)(j + 1) * sd;
    double* cur = w0;
    double* other = w1;
    for (int64_t n = 0; n < k; ++n) {
        if (a->nst == 1) {
            dst[0] = other;
            forward_step(a, cur, dst.data());
            std::swap(cur, other);
        } else {
            dst[a->nst - 1] = cur;   // the last stage writes U^{n+1} over U^n
            forward_step(a, cur, dst.data());
        }
        ++a->recomputed;
    }
    return cur;
}

// Recompute the stage states of the step that starts from U (stages[0] = U) and reverse it.
static void recompute_and_reverse(fv_adjoint* a, const double* U, int& cur)
{
    const size_t sd = a->state_doubles;
    std::vector<const double*> stages(a->nst);
    stages[0] = U;
    if (a->nst > 1) {
        std::vector<double*> dst(a->nst);
        for (int j = 0; j < a->nst - 1; ++j) dst[j] = a->seg + (size_t)(j + 1) * sd;
        // U^{n+1} itself is not needed: it goes to the second work state
        dst[a->nst - 1] = a->seg + (size_t)(a->nst + 1) * sd;
        forward_step(a, U, dst.data());
        ++a->recomputed;
        for (int j = 1; j < a->nst; ++j) stages[j] = dst[j - 1];
    }
    reverse_step(a, stages.data(), cur);
}

// Reverse steps [n0, n1) from the stored state U_{n0} with s free snapshot slots (slots
// 0..s-1 of a->snap are free).
static void revolve(fv_adjoint* a, int64_t n0, int64_t n1, int64_t s, const double* base, int& cur)
{
    const int64_t l = n1 - n0;
    const size_t sd = a->state_doubles;
    if (l == 1) {
        recompute_and_reverse(a, base, cur);
        return;
    }
    if (s == 0) {
        // with several stages advance() leaves its result in the first work state, and the
        // stage recomputation writes only the stage slots and the second
        for (int64_t k = n1 - 1; k >= n0; --k) recompute_and_reverse(a, advance(a, base, k - n0), cur);
        return;
    }
    const int64_t m = binomial_split(l, s);
    double* slot = a->snap + (size_t)(s - 1) * sd;
    const double* U = advance(a, base, m);
    hipMemcpyAsync(slot, U, sizeof(double) * sd, hipMemcpyDeviceToDevice, a->s->stream);
    revolve(a, n0 + m, n1, s - 1, slot, cur);
    revolve(a, n0, n0 + m, s, base, cur);
}

extern "C" fv_status fv_adjoint_backward(fv_adjoint* a, const double* dQ_dUT, double* dQ_dU0)
{
    if (!a || !dQ_dUT || !dQ_dU0) return fail(FV_EINVAL, "NULL argument");
    if (!a->forward_done) return fail(FV_EINVAL, "fv_adjoint_forward must run first");
    fv_solver* s = a->s;
    HIP_TRY(hipSetDevice(s->device));
    fv_status e = stream_enter(s);
    if (e) return e;
    hipStream_t st = s->stream;
    const size_t sb = sizeof(double) * a->state_doubles;
    const size_t sd = a->state_doubles;
    const int S = a->nst;
    int cur = 0;   // lam[cur] holds dQ/dU^{n+1}
    HIP_TRY(hipMemcpyAsync(a->lam[cur], dQ_dUT, sb, hipMemcpyDeviceToDevice, st));
    a->recomputed = 0;
    a->rev_launch = 0;   // both schedules reverse the steps last to first: same salts
    if (a->binomial) {
        revolve(a, 0, a->nsteps, a->snapshots, a->ckpt, cur);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(dQ_dU0, a->lam[cur], sb, hipMemcpyDeviceToDevice, st));
        HIP_TRY(hipStreamSynchronize(st));
        return stream_leave(s);
    }
    auto slot = [&](int64_t t, int k) { return a->seg + ((size_t)t * S + k) * sd; };
    for (int64_t sg = a->nseg - 1; sg >= 0; --sg) {
        const int64_t k0 = sg * a->every;
        const int64_t K = std::min(a->every, a->nsteps - k0);
        // recompute the segment, keeping every stage state
        HIP_TRY(hipMemcpyAsync(slot(0, 0), a->ckpt + (size_t)sg * sd, sb, hipMemcpyDeviceToDevice, st));
        std::vector<double*> dst(S);
        for (int64_t t = 0; t < K; ++t) {
            for (int k = 0; k < S - 1; ++k) dst[k] = slot(t, k + 1);
            dst[S - 1] = slot(t + 1, 0);
            forward_step(a, slot(t, 0), dst.data());
            ++a->recomputed;
        }
        // reverse the segment's steps
        std::vector<const double*> stages(S);
        for (int64_t t = K - 1; t >= 0; --t) {
            for (int k = 0; k < S; ++k) stages[k] = slot(t, k);
            reverse_step(a, stages.data(), cur);
        }
        HIP_TRY(hipGetLastError());
    }
    HIP_TRY(hipMemcpyAsync(dQ_dU0, a->lam[cur], sb, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    return stream_leave(s);
}

extern "C" fv_status fv_qoi_kinetic_energy(fv_solver* s, const double* state, int64_t batch,
                                           int64_t j0, int64_t j1, const double* seed, double* Q,
                                           double* dQ_dU)
{
    if (!s || !state) return fail(FV_EINVAL, "NULL argument");
    if (s->eq.kind != FV_EQ_EULER) return fail(FV_ENOTSUP, "kinetic energy needs the Euler equations");
    if (batch < 1 || batch > 65535) return fail(FV_EINVAL, "batch must be in [1, 65535]");
    if (j0 < 0 || j1 < j0 || j1 > s->grid.n[1]) return fail(FV_EINVAL, "band outside the grid");
    if (dQ_dU && !seed) return fail(FV_EINVAL, "the gradient needs a seed");
    HIP_TRY(hipSetDevice(s->device));
    const int nblk = qoi_blocks(s->cells);
    fv_status e = ensure_scratch(s, sizeof(double) * (size_t)nblk * batch);
    if (e) return e;
    e = stream_enter(s);
    if (e) return e;
    double volume = 1.0;
    for (int k = 0; k < s->grid.dim; ++k) volume = volume * ((s->grid.hi[k] - s->grid.lo[k]) / (double)s->grid.n[k]);
    const int32_t n32[3] = {(int32_t)s->grid.n[0], (int32_t)s->grid.n[1], (int32_t)s->grid.n[2]};
    launch_qoi_ke(state, s->grid.dim, n32, (int32_t)batch, (int32_t)j0, (int32_t)j1, volume, seed, Q,
                  dQ_dU, (double*)s->scratch, nblk, s->stream);
    HIP_TRY(hipGetLastError());
    return stream_leave(s);
}

extern "C" fv_status fv_line_vjp(fv_solver* s, const double* lambda0, const double* dU_dline,
                                 const double* dline_dtheta, int32_t ntheta, int64_t batch,
                                 double* out)
{
    if (!s || !lambda0 || !dU_dline || !dline_dtheta || !out) return fail(FV_EINVAL, "NULL argument");
    if (ntheta < 1 || batch < 1) return fail(FV_EINVAL, "ntheta and batch must be >= 1");
    if (s->grid.dim < 2) return fail(FV_EINVAL, "lines run along axis 1: dim must be >= 2");
    HIP_TRY(hipSetDevice(s->device));
    const int64_t lines = s->grid.n[0] * s->grid.n[2];
    fv_status e = ensure_scratch(s, sizeof(double) * (size_t)(lines * batch));
    if (e) return e;
    e = stream_enter(s);
    if (e) return e;
    const int32_t n32[3] = {(int32_t)s->grid.n[0], (int32_t)s->grid.n[1], (int32_t)s->grid.n[2]};
    launch_line_vjp(lambda0, dU_dline, dline_dtheta, s->nf, n32, (int32_t)batch, ntheta,
                    (double*)s->scratch, out, s->stream);
    HIP_TRY(hipGetLastError());
    return stream_leave(s);
}
