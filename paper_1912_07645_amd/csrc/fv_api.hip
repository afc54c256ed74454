// fv_api.hip -- host side of libfv: the C ABI declared in include/fv.h.
//
// Time stepping runs without host round trips: per-sample dt, time, step count and status
// live in device memory (fv_control.hip), so a chunk of steps (Runge--Kutta stage launches
// followed by the step-control launch) is captured once into a HIP graph and replayed; the
// host reads back a single counter of running samples after each replay.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/fv.h"
#include "fv_common.h"
#include "fv_control.h"
#include "fv_host.h"
#include <climits>
#include "fv_registry.h"
#include "fv_stats.h"

using namespace fvk;

thread_local std::string g_last_error;

// ------------------------------------------------------------------ errors

extern "C" const char* fv_last_error(void) { return g_last_error.c_str(); }
extern "C" const char* fv_version(void) { return "libfv 0.1 (gfx950)"; }

// ------------------------------------------------------------------ registry

namespace fvk {

static std::vector<RegEntry>& registry()
{
    static std::vector<RegEntry> reg;
    static std::once_flag once;
    std::call_once(once, [] {
        const RegEntry* (*units[])(int*) = {unit_euler1d, unit_euler2d, unit_euler2d_hot,
                                            unit_euler3d, unit_euler3d_hot, unit_scalar1d,
                                            unit_scalar2d, unit_scalar3d, unit_more1d,
                                            unit_more2d, unit_more3d, unit_swe, unit_godunov,
                                            unit_ec, unit_mhd};
        for (auto u : units) {
            int n = 0;
            const RegEntry* t = u(&n);
            reg.insert(reg.end(), t, t + n);
        }
    });
    return reg;
}

int num_stage_variants(int dim, int eq, int recon, int flux)
{
    int n = 0;
    for (const RegEntry& e : registry())
        if (e.dim == dim && e.eq == eq && e.recon == recon && e.flux == flux) ++n;
    return n;
}

const StageKernel* find_stage_kernel(int dim, int eq, int recon, int flux, int variant)
{
    int n = 0;
    for (const RegEntry& e : registry())
        if (e.dim == dim && e.eq == eq && e.recon == recon && e.flux == flux) {
            if (n == variant) return &e.k;
            ++n;
        }
    return nullptr;
}

}  // namespace fvk

// ------------------------------------------------------------------ solver

struct fv_stats {
    const fv_solver* s;
    int32_t max_h;
    int32_t nq;
    int64_t count;
    double* mean = nullptr;
    double* m2 = nullptr;
    double* s2mean = nullptr;
    double* s2m2 = nullptr;
    double* qbuf = nullptr;     // quantities of a chunk of samples
    double* partial = nullptr;  // structure-function partial sums of a chunk
    int32_t chunk;
};

struct WsLayout {
    size_t stage[2];
    size_t dt, mbits, steps, running, active, bad, err, t, count;
    size_t total;
};

static WsLayout ws_layout(const fv_solver* s, int64_t batch)
{
    WsLayout L{};
    size_t off = 0;
    const size_t state_bytes = align256(sizeof(double) * (size_t)batch * s->nf * s->cells);
    for (int i = 0; i < 2; ++i) {
        L.stage[i] = off;
        if (i < n_stage_buffers(s->integ)) off += state_bytes;
    }
    auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
    L.dt = take(sizeof(double) * batch);
    L.mbits = take(sizeof(unsigned long long) * kSpeedSlots * speed_pitch(batch));
    L.steps = take(sizeof(int64_t) * batch);
    L.running = take(sizeof(int32_t) * batch);
    L.active = take(sizeof(int32_t) * batch);
    L.bad = take(sizeof(int32_t) * batch);
    L.err = take(sizeof(int32_t) * batch);
    L.t = take(sizeof(double) * batch);
    L.count = take(sizeof(int32_t) * (1 + kMaxGroups));
    L.total = off;
    return L;
}

static fv_status check_device()
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(FV_EDEVICE, std::string("libfv is built for gfx950, current device is ") + prop.gcnArchName);
    return FV_OK;
}

static fv_status validate_grid(const fv_grid* g)
{
    if (!g) return fail(FV_EINVAL, "grid is NULL");
    if (g->dim < 1 || g->dim > 3) return fail(FV_EINVAL, "grid.dim must be 1, 2 or 3");
    int64_t cells = 1;
    for (int k = 0; k < 3; ++k) {
        if (g->n[k] < 1) return fail(FV_EINVAL, "grid.n must be >= 1 on every axis");
        if (k >= g->dim && g->n[k] != 1) return fail(FV_EINVAL, "grid.n must be 1 beyond grid.dim");
        if (g->n[k] > (1 << 30)) return fail(FV_EINVAL, "grid.n too large");
        if (k < g->dim && !(g->hi[k] > g->lo[k])) return fail(FV_EINVAL, "grid.hi must exceed grid.lo");
        if (g->bc[k] != FV_BC_PERIODIC && g->bc[k] != FV_BC_TRANSMISSIVE)
            return fail(FV_EINVAL, "grid.bc must be periodic or transmissive");
        cells *= g->n[k];
    }
    // cell indices within one sample are 32-bit in the kernels
    if (cells > INT32_MAX) return fail(FV_EINVAL, "grid has more than 2^31 - 1 cells");
    return FV_OK;
}

// Workspace of fv_advance_noalloc: Runge--Kutta stage copies and per-sample control words,
// one copy per device for the life of the process. In host code the array's name stands for
// no device address: kernels and copies take the address that hipGetSymbolAddress returns for
// the current device, kept in noalloc_ptr by fv_create.
constexpr size_t kNoAllocBytes = (size_t)68 << 20;
static __device__ __align__(256) unsigned char noalloc_scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
static std::mutex noalloc_mu;
static void* noalloc_ptr[kMaxDevices];

// Resolve the array's address on `device` (current) once; fv_create calls this.
static fv_status noalloc_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return fail(FV_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(noalloc_mu);
    if (noalloc_ptr[device]) return FV_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch));
    if (e != hipSuccess || !p)
        return fail(FV_EDEVICE, std::string("hipGetSymbolAddress(noalloc_scratch): ") + hipGetErrorString(e));
    noalloc_ptr[device] = p;
    return FV_OK;
}

extern "C" fv_status fv_create(const fv_grid* grid, const fv_equation* eq, int32_t flux,
                               int32_t recon, int32_t integrator, fv_solver** out)
{
    if (!out) return fail(FV_EINVAL, "out is NULL");
    *out = nullptr;
    fv_status st = validate_grid(grid);
    if (st) return st;
    if (!eq) return fail(FV_EINVAL, "equation is NULL");
    if (eq->kind < 0 || eq->kind > 4) return fail(FV_EINVAL, "unknown equation kind");
    if (eq->kind == FV_EQ_SHALLOW_WATER) {
        if (!(eq->gravity > 0.0) || !std::isfinite(eq->gravity)) return fail(FV_EINVAL, "gravity must be positive");
        if (grid->dim > 2) return fail(FV_ENOTSUP, "the shallow-water equations are offered in 1D and 2D");
    }
    if (flux < 0 || flux > 6) return fail(FV_EINVAL, "unknown flux");
    if (recon < 0 || recon > 3) return fail(FV_EINVAL, "unknown reconstruction");
    if ((flux == FV_FLUX_EC || flux == FV_FLUX_EC4) && eq->kind != FV_EQ_BURGERS && eq->kind != FV_EQ_EULER)
        return fail(FV_ENOTSUP, "the entropy-conservative fluxes are offered for Burgers and Euler");
    if (flux == FV_FLUX_EC4 && recon != FV_RECON_FIRST_ORDER)
        return fail(FV_ENOTSUP, "the fourth-order entropy-conservative flux takes the cell values (first order)");
    if (flux == FV_FLUX_GODUNOV && eq->kind == FV_EQ_SHALLOW_WATER)
        return fail(FV_ENOTSUP, "Godunov's flux is not offered for the shallow-water equations");
    if (integrator < 0 || integrator > 2) return fail(FV_EINVAL, "unknown integrator");
    if (flux == FV_FLUX_HLLC && eq->kind != FV_EQ_EULER)
        return fail(FV_ENOTSUP, "HLLC needs the Euler equations");
    if ((eq->kind == FV_EQ_EULER || eq->kind == FV_EQ_MHD) && !(eq->gamma > 1.0))
        return fail(FV_EINVAL, "gamma must exceed 1");
    if (eq->kind == FV_EQ_MHD && flux != FV_FLUX_RUSANOV && flux != FV_FLUX_HLL)
        return fail(FV_ENOTSUP, "ideal MHD is offered with the Rusanov and HLL fluxes");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(eq->velocity[k])) return fail(FV_EINVAL, "velocity must be finite");
    st = check_device();
    if (st) return st;
    const StageKernel* kern = find_stage_kernel(grid->dim, eq->kind, recon, flux, 0);
    if (!kern) return fail(FV_ENOTSUP, "no kernel for this combination");

    fv_solver* s = new (std::nothrow) fv_solver();
    if (!s) return fail(FV_ENOMEM, "host allocation failed");
    s->grid = *grid;
    s->eq = *eq;
    s->flux = flux;
    s->recon = recon;
    s->integ = integrator;
    s->nf = eq->kind == FV_EQ_EULER ? grid->dim + 2
          : (eq->kind == FV_EQ_SHALLOW_WATER ? grid->dim + 1 : (eq->kind == FV_EQ_MHD ? 8 : 1));
    s->cells = grid->n[0] * grid->n[1] * grid->n[2];
    s->variant = 0;
    s->kern = kern;
    s->ph.gamma = eq->gamma;
    s->ph.gm1 = eq->gamma - 1.0;
    s->ph.grav = eq->gravity;
    for (int k = 0; k < 3; ++k) {
        s->ph.vel[k] = eq->velocity[k];
        s->ph.inv_dx[k] = (double)grid->n[k] / (grid->hi[k] - grid->lo[k]);
    }
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipHostMalloc((void**)&s->host_count, sizeof(int32_t) * (1 + kMaxGroups), hipHostMallocDefault);
    if (e != hipSuccess) {
        fv_destroy(s);
        return fail(FV_EDEVICE, std::string("fv_create: ") + hipGetErrorString(e));
    }
    st = noalloc_setup(s->device);
    if (st) {
        fv_destroy(s);
        return st;
    }
    if (grid->dim == 1) {
        const SmallKernel* sk = find_small_kernel(eq->kind, recon, flux);
        if (sk && grid->n[0] <= sk->max_cells) s->small = sk;
    }
    // The tuner's stored choice for this shape, if any.
    const char* v = std::getenv("FV_VARIANT");
    if (v) {
        int vi = std::atoi(v);
        const StageKernel* k2 = find_stage_kernel(grid->dim, eq->kind, recon, flux, vi);
        if (k2) { s->variant = vi; s->kern = k2; }
        else if (s->small && vi == num_stage_variants(grid->dim, eq->kind, recon, flux)) {
            s->variant = vi;
            s->use_small = true;
        }
    }
    *out = s;
    return FV_OK;
}

extern "C" fv_status fv_destroy(fv_solver* s)
{
    if (!s) return FV_OK;
    if (s->stream) hipStreamSynchronize(s->stream);
    drop_graph(s);
    for (hipEvent_t e : s->prof_ev) hipEventDestroy(e);
    if (s->scratch) hipFree(s->scratch);
    if (s->ws && s->ws_owned) hipFree(s->ws);
    if (s->host_count) hipHostFree(s->host_count);
    if (s->ev) hipEventDestroy(s->ev);
    if (s->stream) hipStreamDestroy(s->stream);
    delete s;
    return FV_OK;
}

extern "C" fv_status fv_set_stream(fv_solver* s, void* stream)
{
    if (!s) return fail(FV_EINVAL, "solver is NULL");
    s->user_stream = (hipStream_t)stream;
    return FV_OK;
}

extern "C" int32_t fv_num_fields(const fv_solver* s) { return s ? s->nf : -1; }

extern "C" fv_status fv_workspace_size(const fv_solver* s, int64_t batch, size_t* bytes)
{
    if (!s || !bytes) return fail(FV_EINVAL, "NULL argument");
    if (batch < 1) return fail(FV_EINVAL, "batch must be >= 1");
    *bytes = ws_layout(s, batch).total;
    return FV_OK;
}

extern "C" fv_status fv_set_workspace(fv_solver* s, void* dev_ptr, size_t bytes)
{
    if (!s) return fail(FV_EINVAL, "solver is NULL");
    if (dev_ptr && ((uintptr_t)dev_ptr & 255)) return fail(FV_EINVAL, "workspace must be 256-byte aligned");
    HIP_TRY(hipStreamSynchronize(s->stream));
    drop_graph(s);
    if (s->ws && s->ws_owned) HIP_TRY(hipFree(s->ws));
    s->ws = dev_ptr;
    s->ws_bytes = dev_ptr ? bytes : 0;
    s->ws_owned = (dev_ptr == nullptr);
    return FV_OK;
}

static fv_status ensure_workspace(fv_solver* s, size_t need)
{
    if (need <= s->ws_bytes && s->ws) return FV_OK;
    if (!s->ws_owned) return fail(FV_ENOMEM, "caller workspace too small for this batch");
    HIP_TRY(hipStreamSynchronize(s->stream));
    drop_graph(s);
    if (s->ws) HIP_TRY(hipFree(s->ws));
    s->ws = nullptr;
    s->ws_bytes = 0;
    void* p = nullptr;
    if (hipMalloc(&p, need) != hipSuccess) return fail(FV_ENOMEM, "workspace allocation failed");
    s->ws = p;
    s->ws_bytes = need;
    return FV_OK;
}

// ------------------------------------------------------------------ one group's pointers

struct GroupRun {
    fv_solver* s;
    double* state;
    int64_t batch;
    double* t;
    int64_t* steps;
    int32_t* err;
    WsLayout L;
    char* ws;
};

static Group make_group(const GroupRun& r, int stage)
{
    const fv_solver* s = r.s;
    Group g{};
    double* st1 = (double*)(r.ws + r.L.stage[0]);
    double* st2 = (double*)(r.ws + r.L.stage[1]);
    const int S = n_stages(s->integ);
    // sources / destinations of each stage (RK3: U^n -> W1 -> W2 -> U^n; RK2: U^n -> W1 -> U^n;
    // forward Euler: U^n -> W1, copied back)
    const double* src = (stage == 0) ? r.state : (stage == 1 ? st1 : st2);
    double* dst;
    if (S == 1) dst = st1;
    else if (stage == S - 1) dst = r.state;
    else dst = (stage == 0) ? st1 : st2;
    g.src = src;
    g.un = r.state;
    g.dst = dst;
    g.dt = (const double*)(r.ws + r.L.dt);
    g.active = (const int32_t*)(r.ws + r.L.active);
    g.mbits = (unsigned long long*)(r.ws + r.L.mbits);
    g.bad = (int32_t*)(r.ws + r.L.bad);
    g.cells = s->cells;
    const int32_t tb[3] = {s->kern->bx, s->kern->by, s->kern->bz};
    g.ntiles = 1;
    for (int k = 0; k < 3; ++k) {
        g.n[k] = (int32_t)s->grid.n[k];
        g.tiles[k] = (int32_t)((s->grid.n[k] + tb[k] - 1) / tb[k]);
        g.ntiles *= g.tiles[k];
    }
    g.batch = (int32_t)r.batch;
    g.ph = s->ph;
    return g;
}

static CtrlGroup make_ctrl(const GroupRun& r)
{
    CtrlGroup c{};
    c.t = r.t ? r.t : (double*)(r.ws + r.L.t);
    c.dt = (double*)(r.ws + r.L.dt);
    c.running = (int32_t*)(r.ws + r.L.running);
    c.active = (int32_t*)(r.ws + r.L.active);
    c.mbits = (unsigned long long*)(r.ws + r.L.mbits);
    c.bad = (int32_t*)(r.ws + r.L.bad);
    c.steps = r.steps ? r.steps : (int64_t*)(r.ws + r.L.steps);
    c.err = r.err ? r.err : (int32_t*)(r.ws + r.L.err);
    c.batch = (int32_t)r.batch;
    return c;
}

struct StepPlan {
    std::vector<StageArgs> stages;
    CopyArgs copy{};
    bool copy_back = false;
    CtrlArgs ctrl{};
    SpeedArgs speed{};
    const StageKernel* kern = nullptr;
};

static StepPlan make_plan(std::vector<GroupRun>& runs)
{
    StepPlan p;
    const fv_solver* s0 = runs[0].s;
    p.kern = s0->kern;
    const int S = n_stages(s0->integ);
    for (int st = 0; st < S; ++st) {
        StageArgs a{};
        a.ngroups = (int32_t)runs.size();
        int64_t blocks = 0;
        for (size_t i = 0; i < runs.size(); ++i) {
            a.g[i] = make_group(runs[i], st);
            a.g[i].block0 = blocks;
            blocks += (int64_t)a.g[i].ntiles * a.g[i].batch;
        }
        for (int k = 0; k < 3; ++k) a.bc[k] = s0->grid.bc[k];
        a.beta = stage_beta(s0->integ, st);
        a.use_un = st > 0;
        a.last = (st == S - 1);
        a.nblocks = blocks;
        p.stages.push_back(a);
    }
    if (S == 1) {
        p.copy_back = true;
        p.copy.ngroups = (int32_t)runs.size();
        for (size_t i = 0; i < runs.size(); ++i) {
            CopyGroup& c = p.copy.g[i];
            c.src = (const double*)(runs[i].ws + runs[i].L.stage[0]);
            c.dst = runs[i].state;
            c.active = (const int32_t*)(runs[i].ws + runs[i].L.active);
            c.per_sample = (int64_t)runs[i].s->nf * runs[i].s->cells;
            c.batch = (int32_t)runs[i].batch;
        }
    }
    p.ctrl.ngroups = (int32_t)runs.size();
    for (size_t i = 0; i < runs.size(); ++i) p.ctrl.g[i] = make_ctrl(runs[i]);
    p.ctrl.n_running = (int32_t*)(runs[0].ws + runs[0].L.count);
    p.speed.ngroups = (int32_t)runs.size();
    int64_t blocks = 0;
    for (size_t i = 0; i < runs.size(); ++i) {
        Group g = make_group(runs[i], 0);
        g.src = runs[i].state;
        g.block0 = blocks;
        const int64_t per = (runs[i].s->cells + p.kern->cells_per_block - 1) / p.kern->cells_per_block;
        blocks += per * runs[i].batch;
        p.speed.g[i] = g;
    }
    p.speed.nblocks = blocks;
    return p;
}

// With ev (profiling), the step's stage launches, which follow each other directly, are
// bracketed by one pair of events: ev[0] before the first, ev[1] after the last.
static void enqueue_step(const StepPlan& p, hipStream_t st, hipEvent_t* ev = nullptr)
{
    if (ev) hipEventRecord(ev[0], st);
    for (const StageArgs& a : p.stages) p.kern->stage(a, st);
    if (ev) hipEventRecord(ev[1], st);
    if (p.copy_back) launch_copy_back(p.copy, st);
    launch_ctrl_begin(p.ctrl, st);
}

// FV_NO_GRAPH=1 enqueues every launch eagerly instead of replaying a captured graph.
static bool graphs_enabled()
{
    const char* e = std::getenv("FV_NO_GRAPH");
    return !(e && e[0] && e[0] != '0');
}

// Chunk of steps per graph replay.
static int64_t chunk_steps(int64_t max_steps)
{
    const char* e = std::getenv("FV_CHUNK");
    int64_t c = e ? std::max<long long>(1, std::atoll(e)) : 16;
    return std::min<int64_t>(c, std::max<int64_t>(1, max_steps));
}

// Step-control settings of a run (copied into every plan).
struct CtrlParams {
    int32_t fixed, limit_is_error;
    double t_end, cfl, fixed_dt, cfl_bound;
    int64_t max_steps;
};

static void apply_params(StepPlan& p, const CtrlParams& c)
{
    p.ctrl.fixed = c.fixed;
    p.ctrl.limit_is_error = c.limit_is_error;
    p.ctrl.t_end = c.t_end;
    p.ctrl.cfl = c.cfl;
    p.ctrl.fixed_dt = c.fixed_dt;
    p.ctrl.cfl_bound = c.cfl_bound;
    p.ctrl.max_steps = c.max_steps;
}

// Run the step loop until no sample is running. When a group (a grid of a multi-group run)
// has no running sample left, it is dropped from the launches and the graph is captured
// again, so finished coarse levels stop costing launch slots.
static fv_status run_steps(fv_solver* s0, std::vector<GroupRun> runs, const CtrlParams& cp,
                           const std::vector<char>& key0, bool eager_only = false)
{
    hipStream_t st = s0->stream;
    const int64_t max_steps = cp.max_steps;
    StepPlan p = make_plan(runs);
    apply_params(p, cp);
    int32_t* counts_dev = p.ctrl.n_running;
    launch_ctrl_reset(p.ctrl, st);
    p.kern->speed(p.speed, st);
    launch_ctrl_begin(p.ctrl, st);
    HIP_TRY(hipGetLastError());
    const int64_t chunk = chunk_steps(max_steps);
    const bool profile = s0->profile && !eager_only;
    const bool use_graph = graphs_enabled() && !profile && !eager_only;
    const size_t nst = p.stages.size();
    if (profile) {
        const size_t need = 2 * (size_t)chunk;
        while (s0->prof_ev.size() < need) {
            hipEvent_t e;
            HIP_TRY(hipEventCreate(&e));
            s0->prof_ev.push_back(e);
        }
    }
    std::vector<char> key = key0;
    auto read_counts = [&]() -> fv_status {
        HIP_TRY(hipMemcpyAsync(s0->host_count, counts_dev, sizeof(int32_t) * (1 + runs.size()),
                               hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        return FV_OK;
    };
    fv_status e = read_counts();
    if (e) return e;
    if (s0->host_count[0] == 0) return FV_OK;
    int64_t done = 0;
    while (done < max_steps) {
        // drop groups that have finished (multi-group runs only)
        if (runs.size() > 1) {
            std::vector<GroupRun> keep;
            for (size_t i = 0; i < runs.size(); ++i)
                if (s0->host_count[1 + i] > 0) keep.push_back(runs[i]);
            if (keep.size() != runs.size()) {
                runs = keep;
                p = make_plan(runs);
                apply_params(p, cp);
                p.ctrl.n_running = counts_dev;
                drop_graph(s0);
                key.push_back((char)runs.size());
            }
        }
        if (use_graph && (s0->graph.key != key || !s0->graph.exec)) {
            drop_graph(s0);
            hipGraph_t g = nullptr;
            HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            for (int64_t i = 0; i < chunk; ++i) enqueue_step(p, st);
            hipError_t ce = hipStreamEndCapture(st, &g);
            if (ce != hipSuccess) return fail(FV_EDEVICE, std::string("graph capture: ") + hipGetErrorString(ce));
            ce = hipGraphInstantiate(&s0->graph.exec, g, nullptr, nullptr, 0);
            hipGraphDestroy(g);
            if (ce != hipSuccess) return fail(FV_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(ce));
            s0->graph.key = key;
        }
        // Each round advances every running sample by up to `chunk` steps (a captured graph),
        // or by the remaining max_steps % chunk steps (enqueued directly) once fewer than
        // `chunk` remain, so a run limited by max_steps launches exactly max_steps steps. A
        // sample stops at t_end, on an error or at max_steps; after max_steps steps none runs.
        const int64_t n = std::min<int64_t>(chunk, std::max<int64_t>(1, max_steps - done));
        if (use_graph && n == chunk) {
            HIP_TRY(hipGraphLaunch(s0->graph.exec, st));
        } else {
            for (int64_t i = 0; i < n; ++i)
                enqueue_step(p, st, profile ? &s0->prof_ev[2 * (size_t)i] : nullptr);
            HIP_TRY(hipGetLastError());
        }
        done += n;
        e = read_counts();
        if (e) return e;
        if (profile) {
            for (size_t i = 0; i < (size_t)n; ++i) {
                float ms = 0.0f;
                HIP_TRY(hipEventElapsedTime(&ms, s0->prof_ev[2 * i], s0->prof_ev[2 * i + 1]));
                s0->prof_stage_ms += ms;
                s0->prof_stage_launches += (int64_t)nst;
            }
        }
        if (s0->host_count[0] == 0) return FV_OK;
    }
    return fail(FV_EDEVICE, "step loop did not terminate");
}

static fv_status first_error(fv_solver* s, const int32_t* err_dev, int64_t batch, fv_status* out)
{
    std::vector<int32_t> h((size_t)batch);
    HIP_TRY(hipMemcpyAsync(h.data(), err_dev, sizeof(int32_t) * batch, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    *out = FV_OK;
    for (int64_t b = 0; b < batch; ++b)
        if (h[b] != 0) {
            *out = (fv_status)h[b];
            g_last_error = "sample " + std::to_string(b) + " failed with status " + std::to_string(h[b]);
            break;
        }
    return FV_OK;
}

template <class T>
static void key_push(std::vector<char>& k, const T& v)
{
    const char* p = (const char*)&v;
    k.insert(k.end(), p, p + sizeof(T));
}

// fixed_ws (with fixed_ws_bytes): run in this device memory instead of the solver's workspace,
// with the tiled kernels launched eagerly (no graph, no timing events) and the first failing
// sample found on the device, so that the call allocates nothing.
static fv_status evolve_common(fv_solver* s, double* state, int64_t batch, double* t,
                               double t_end, double cfl, int64_t max_steps, int64_t* steps,
                               int32_t* err, bool limit_is_error, bool fixed, double fixed_dt,
                               double cfl_bound, char* fixed_ws = nullptr,
                               size_t fixed_ws_bytes = 0)
{
    if (!s) return fail(FV_EINVAL, "solver is NULL");
    if (!state) return fail(FV_EINVAL, "state is NULL");
    if (batch < 1 || batch > (1 << 24)) return fail(FV_EINVAL, "batch must be in [1, 2^24]");
    if (!fixed) {
        if (!t) return fail(FV_EINVAL, "t is NULL");
        if (!(cfl > 0.0) || cfl > 1.0) return fail(FV_EINVAL, "cfl must be in (0, 1]");
        if (!std::isfinite(t_end)) return fail(FV_EINVAL, "t_end must be finite");
    } else {
        if (!(fixed_dt > 0.0) || !std::isfinite(fixed_dt)) return fail(FV_EINVAL, "dt must be > 0");
        if (!(cfl_bound > 0.0)) return fail(FV_EINVAL, "cfl_bound must be > 0");
    }
    if (max_steps < 0) return fail(FV_EINVAL, "max_steps must be >= 0");
    const int64_t blocks_per_sample = [&] {
        int64_t n = 1;
        const int32_t tb[3] = {s->kern->bx, s->kern->by, s->kern->bz};
        for (int k = 0; k < 3; ++k) n *= (s->grid.n[k] + tb[k] - 1) / tb[k];
        return n;
    }();
    if (blocks_per_sample * batch > 0x7fffffffLL) return fail(FV_EINVAL, "launch too large");
    HIP_TRY(hipSetDevice(s->device));
    if (s->use_small && !s->profile && !fixed_ws) {
        // the single-workgroup time loop: each launch runs every sample up to kSmallChunk
        // steps; launches repeat while samples still run
        constexpr int64_t kSmallChunk = 1 << 16;
        const size_t nb = (size_t)batch;
        // scratch: running flags, the running count, and step counts / status where the
        // caller passes none
        const size_t off_count = sizeof(int32_t) * nb;
        const size_t off_steps = (off_count + sizeof(int32_t) + 7) & ~(size_t)7;
        const size_t off_err = off_steps + sizeof(int64_t) * nb;
        fv_status st = ensure_scratch(s, off_err + sizeof(int32_t) * nb);
        if (st) return st;
        st = stream_enter(s);
        if (st) return st;
        char* sc = (char*)s->scratch;
        SmallArgs a{};
        a.state = state;
        a.batch = batch;
        a.n = (int32_t)s->grid.n[0];
        a.bc = s->grid.bc[0];
        a.ph = s->ph;
        a.t = fixed ? nullptr : t;
        a.steps = steps ? steps : (int64_t*)(sc + off_steps);
        a.err = err ? err : (int32_t*)(sc + off_err);
        a.running = (int32_t*)sc;
        a.n_running = (int32_t*)(sc + off_count);
        a.chunk = kSmallChunk;
        a.t_end = t_end;
        a.cfl = cfl;
        a.max_steps = max_steps;
        a.limit_is_error = limit_is_error ? 1 : 0;
        a.fixed = fixed ? 1 : 0;
        a.fixed_dt = fixed_dt;
        a.cfl_bound = cfl_bound;
        a.nst = n_stages(s->integ);
        for (int k = 0; k < a.nst; ++k) a.beta[k] = stage_beta(s->integ, k);
        for (a.first = 1;; a.first = 0) {
            HIP_TRY(hipMemsetAsync(a.n_running, 0, sizeof(int32_t), s->stream));
            s->small->launch(a, s->stream);
            HIP_TRY(hipGetLastError());
            HIP_TRY(hipMemcpyAsync(s->host_count, a.n_running, sizeof(int32_t), hipMemcpyDeviceToHost,
                                   s->stream));
            HIP_TRY(hipStreamSynchronize(s->stream));
            if (s->host_count[0] == 0) break;
        }
        fv_status result = FV_OK;
        st = first_error(s, a.err, batch, &result);
        if (st) return st;
        st = stream_leave(s);
        if (st) return st;
        return result;
    }
    WsLayout L = ws_layout(s, batch);
    fv_status st = FV_OK;
    if (fixed_ws) {
        if (L.total > fixed_ws_bytes)
            return fail(FV_ENOMEM, "batch needs " + std::to_string(L.total) +
                                       " bytes of workspace; the allocation-free call has " +
                                       std::to_string(fixed_ws_bytes));
    } else {
        st = ensure_workspace(s, L.total);
        if (st) return st;
    }
    st = stream_enter(s);
    if (st) return st;
    char* ws = fixed_ws ? fixed_ws : (char*)s->ws;

    std::vector<GroupRun> runs{GroupRun{s, state, batch, fixed ? nullptr : t, steps, err, L, ws}};
    const CtrlParams cp{fixed ? 1 : 0, limit_is_error ? 1 : 0, t_end, cfl, fixed_dt, cfl_bound, max_steps};

    std::vector<char> key;
    key_push(key, state); key_push(key, batch); key_push(key, t); key_push(key, steps);
    key_push(key, err); key_push(key, t_end); key_push(key, cfl); key_push(key, max_steps);
    key_push(key, limit_is_error); key_push(key, fixed); key_push(key, fixed_dt);
    key_push(key, cfl_bound); key_push(key, s->ws); key_push(key, s->variant);
    key_push(key, chunk_steps(max_steps));

    st = run_steps(s, runs, cp, key, fixed_ws != nullptr);
    if (st) return st;
    fv_status result = FV_OK;
    if (fixed_ws) {
        // the first failing sample, found on the device and read into the pinned counters
        launch_first_error(make_ctrl(runs[0]).err, (int32_t)batch, (int32_t*)(ws + L.count), s->stream);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(s->host_count, ws + L.count, 2 * sizeof(int32_t),
                               hipMemcpyDeviceToHost, s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
        if (s->host_count[0] != 0) {
            result = (fv_status)s->host_count[0];
            g_last_error = "sample " + std::to_string(s->host_count[1]) + " failed with status " +
                           std::to_string(s->host_count[0]);
        }
    } else {
        st = first_error(s, make_ctrl(runs[0]).err, batch, &result);
        if (st) return st;
    }
    st = stream_leave(s);
    if (st) return st;
    return result;
}

extern "C" fv_status fv_evolve(fv_solver* s, double* state, int64_t batch, double* t, double t_end,
                               double cfl, int64_t max_steps, int64_t* steps, int32_t* err)
{
    return evolve_common(s, state, batch, t, t_end, cfl, max_steps, steps, err, true, false, 0.0, 0.0);
}

extern "C" fv_status fv_advance(fv_solver* s, double* state, int64_t batch, double* t, double t_end,
                                double cfl, int64_t nsteps, int64_t* steps, int32_t* err)
{
    return evolve_common(s, state, batch, t, t_end, cfl, nsteps, steps, err, false, false, 0.0, 0.0);
}

// ------------------------------------------------------------------ allocation-free stepping

extern "C" size_t fv_noalloc_capacity(void) { return kNoAllocBytes; }

extern "C" fv_status fv_advance_noalloc(fv_solver* s, double* state, int64_t batch, double* t,
                                        double t_end, double cfl, int64_t nsteps, int64_t* steps,
                                        int32_t* err)
{
    if (!s) return fail(FV_EINVAL, "solver is NULL");
    void* p = nullptr;
    {
        std::lock_guard<std::mutex> lock(noalloc_mu);
        if (s->device >= 0 && s->device < kMaxDevices) p = noalloc_ptr[s->device];
    }
    if (!p) return fail(FV_EDEVICE, "no allocation-free workspace on the solver's device");
    return evolve_common(s, state, batch, t, t_end, cfl, nsteps, steps, err, false, false, 0.0, 0.0,
                         (char*)p, kNoAllocBytes);
}

extern "C" fv_status fv_evolve_fixed_dt(fv_solver* s, double* state, int64_t batch, double dt,
                                        int64_t nsteps, double cfl_bound, int32_t* err)
{
    return evolve_common(s, state, batch, nullptr, 0.0, 1.0, nsteps, nullptr, err, false, true, dt,
                         cfl_bound);
}

extern "C" fv_status fv_evolve_multi(int32_t n_groups, fv_solver* const* solvers,
                                     double* const* states, const int64_t* batches,
                                     double* const* t, double t_end, double cfl,
                                     int64_t max_steps, int64_t* const* steps,
                                     int32_t* const* err)
{
    if (n_groups < 1 || n_groups > kMaxGroups) return fail(FV_EINVAL, "n_groups must be in [1, 8]");
    if (!solvers || !states || !batches || !t) return fail(FV_EINVAL, "NULL argument");
    if (!(cfl > 0.0) || cfl > 1.0) return fail(FV_EINVAL, "cfl must be in (0, 1]");
    if (max_steps < 0) return fail(FV_EINVAL, "max_steps must be >= 0");
    fv_solver* s0 = solvers[0];
    if (!s0) return fail(FV_EINVAL, "solver is NULL");
    for (int i = 0; i < n_groups; ++i) {
        const fv_solver* s = solvers[i];
        if (!s || !states[i] || !t[i]) return fail(FV_EINVAL, "NULL solver, state or t");
        if (batches[i] < 1) return fail(FV_EINVAL, "batches must be >= 1");
        if (s->grid.dim != s0->grid.dim || s->eq.kind != s0->eq.kind || s->flux != s0->flux ||
            s->recon != s0->recon || s->integ != s0->integ || s->kern != s0->kern)
            return fail(FV_EINVAL, "solvers must share dimension, equation, scheme and tile");
        for (int k = 0; k < 3; ++k)
            if (s->grid.bc[k] != s0->grid.bc[k]) return fail(FV_EINVAL, "solvers must share boundary conditions");
        for (int j = 0; j < i; ++j)
            if (solvers[j] == s) return fail(FV_EINVAL, "each group needs its own solver");
    }
    HIP_TRY(hipSetDevice(s0->device));
    std::vector<GroupRun> runs;
    for (int i = 0; i < n_groups; ++i) {
        fv_solver* s = solvers[i];
        WsLayout L = ws_layout(s, batches[i]);
        fv_status st = ensure_workspace(s, L.total);
        if (st) return st;
        runs.push_back(GroupRun{s, states[i], batches[i], t[i], steps ? steps[i] : nullptr,
                                err ? err[i] : nullptr, L, (char*)s->ws});
    }
    fv_status st = stream_enter(s0);
    if (st) return st;
    const CtrlParams cp{0, 1, t_end, cfl, 0.0, 0.0, max_steps};
    std::vector<char> key;
    key_push(key, n_groups);
    for (int i = 0; i < n_groups; ++i) {
        key_push(key, solvers[i]); key_push(key, states[i]); key_push(key, batches[i]);
        key_push(key, t[i]); key_push(key, err ? err[i] : nullptr); key_push(key, solvers[i]->ws);
        key_push(key, steps ? steps[i] : nullptr);
    }
    key_push(key, t_end); key_push(key, cfl); key_push(key, max_steps); key_push(key, s0->variant);
    key_push(key, chunk_steps(max_steps));
    st = run_steps(s0, runs, cp, key);
    if (st) return st;
    fv_status result = FV_OK;
    for (int i = 0; i < n_groups && result == FV_OK; ++i) {
        st = first_error(s0, make_ctrl(runs[i]).err, batches[i], &result);
        if (st) return st;
    }
    st = stream_leave(s0);
    if (st) return st;
    return result;
}

// ------------------------------------------------------------------ kernel timing

extern "C" fv_status fv_profile_enable(fv_solver* s, int32_t on)
{
    if (!s) return fail(FV_EINVAL, "solver is NULL");
    s->profile = on != 0;
    s->prof_stage_ms = 0.0;
    s->prof_stage_launches = 0;
    return FV_OK;
}

extern "C" fv_status fv_profile_read(const fv_solver* s, double* stage_ms, int64_t* stage_launches)
{
    if (!s) return fail(FV_EINVAL, "solver is NULL");
    if (stage_ms) *stage_ms = s->prof_stage_ms;
    if (stage_launches) *stage_launches = s->prof_stage_launches;
    return FV_OK;
}

// ------------------------------------------------------------------ tuner

extern "C" int32_t fv_num_variants(const fv_solver* s)
{
    if (!s) return -1;
    return num_stage_variants(s->grid.dim, s->eq.kind, s->recon, s->flux) + (s->small ? 1 : 0);
}

extern "C" fv_status fv_set_variant(fv_solver* s, int32_t variant)
{
    if (!s) return fail(FV_EINVAL, "solver is NULL");
    const StageKernel* k = find_stage_kernel(s->grid.dim, s->eq.kind, s->recon, s->flux, variant);
    const bool small = !k && s->small &&
                       variant == num_stage_variants(s->grid.dim, s->eq.kind, s->recon, s->flux);
    if (!k && !small) return fail(FV_EINVAL, "no such variant");
    HIP_TRY(hipStreamSynchronize(s->stream));
    drop_graph(s);
    s->variant = variant;
    s->use_small = small;
    if (k) s->kern = k;   // the single-workgroup variant keeps the tiled kernel for other calls
    return FV_OK;
}

extern "C" fv_status fv_get_tile(const fv_solver* s, int32_t* bx, int32_t* by, int32_t* bz, int32_t* variant)
{
    if (!s) return fail(FV_EINVAL, "solver is NULL");
    if (bx) *bx = s->use_small ? (int32_t)s->grid.n[0] : s->kern->bx;   // one workgroup per sample
    if (by) *by = s->use_small ? 1 : s->kern->by;
    if (bz) *bz = s->use_small ? 1 : s->kern->bz;
    if (variant) *variant = s->variant;
    return FV_OK;
}

// Time runs of whole steps (all Runge--Kutta stages) of every tile variant on `state` for
// `batch` samples and keep the variant with the fastest median run. The state is not
// modified: the tuner evolves a copy in a buffer of its own. Results of every variant are
// bitwise identical, so the choice affects speed only.
extern "C" fv_status fv_tune(fv_solver* s, double* state, int64_t batch, int32_t reps, int32_t* chosen)
{
    if (!s || !state) return fail(FV_EINVAL, "NULL argument");
    if (batch < 1) return fail(FV_EINVAL, "batch must be >= 1");
    const int nv = fv_num_variants(s);
    if (reps < 1) reps = 3;
    HIP_TRY(hipSetDevice(s->device));
    const size_t state_bytes = sizeof(double) * (size_t)batch * s->nf * s->cells;
    double* scratch = nullptr;
    HIP_TRY(hipMalloc((void**)&scratch, align256(state_bytes) + sizeof(double) * batch));
    double* t = (double*)((char*)scratch + align256(state_bytes));
    // one run of n steps on a fresh copy of the state; its wall time in *sec
    auto run = [&](int64_t n, double* sec) -> fv_status {
        if (hipMemcpyAsync(scratch, state, state_bytes, hipMemcpyDeviceToDevice, s->stream) != hipSuccess ||
            hipMemsetAsync(t, 0, sizeof(double) * batch, s->stream) != hipSuccess ||
            hipStreamSynchronize(s->stream) != hipSuccess)
            return fail(FV_EDEVICE, "tuner copy failed");
        auto t0 = std::chrono::steady_clock::now();
        fv_status e = fv_advance(s, scratch, batch, t, 1e300, 0.4, n, nullptr, nullptr);
        auto t1 = std::chrono::steady_clock::now();
        *sec = std::chrono::duration<double>(t1 - t0).count();
        return e;
    };
    const int v0 = s->variant;
    fv_status st = fv_set_variant(s, 0);
    // Steps per timed run: about 8 ms of work (between 4 and 32), the same for every variant.
    // Then about 50 ms of untimed steps, so that the clocks have left their idle state before
    // the first variant is timed (timed cold, the first variant would lose).
    double sec = 0.0;
    int64_t nsteps = 4;
    if (st == FV_OK) st = run(4, &sec);
    if (st == FV_OK) {
        nsteps = std::max<int64_t>(4, std::min<int64_t>(32, (int64_t)(8e-3 / std::max(sec / 4, 1e-9))));
        double warm = 0.0;
        while (st == FV_OK && warm < 50e-3) {
            st = run(nsteps, &sec);
            warm += sec;
        }
    }
    double best = 1e300;
    int best_v = v0;
    for (int v = 0; v < nv && st == FV_OK; ++v) {
        st = fv_set_variant(s, v);
        if (st) break;
        // an untimed run loads the variant's kernels and captures its step graph
        std::vector<double> times;
        for (int r = 0; r < reps + 1 && st == FV_OK; ++r) {
            st = run(nsteps, &sec);
            if (r > 0) times.push_back(sec);
        }
        if (st) break;
        std::sort(times.begin(), times.end());
        const double med = times[times.size() / 2];
        if (med < best) { best = med; best_v = v; }
    }
    hipFree(scratch);
    if (st) {
        fv_set_variant(s, v0);
        return st;
    }
    st = fv_set_variant(s, best_v);
    if (chosen) *chosen = best_v;
    return st;
}

// ------------------------------------------------------------------ arithmetic self-check

__global__ void arith_kernel(const double* a, const double* b, double* quot, double* root, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        quot[i] = a[i] / b[i];
        root[i] = sqrt(a[i]);
    }
}

extern "C" fv_status fv_check_arith(const double* a, const double* b, double* quot, double* root,
                                    int64_t n)
{
    if (!a || !b || !quot || !root || n < 0) return fail(FV_EINVAL, "bad argument");
    if (n == 0) return FV_OK;
    hipLaunchKernelGGL(arith_kernel, dim3(1024), dim3(256), 0, 0, a, b, quot, root, n);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipDeviceSynchronize());
    return FV_OK;
}

// ------------------------------------------------------------------ statistics

extern "C" fv_status fv_stats_create(const fv_solver* s, int32_t max_h, fv_stats** out)
{
    if (!s || !out) return fail(FV_EINVAL, "NULL argument");
    *out = nullptr;
    if (max_h < 0) return fail(FV_EINVAL, "max_h must be >= 0");
    if (max_h > 0)
        for (int k = 0; k < s->grid.dim; ++k)
            if (s->grid.bc[k] != FV_BC_PERIODIC || max_h >= s->grid.n[k])
                return fail(FV_ENOTSUP, "structure functions need periodic axes with max_h < n");
    fv_stats* st = new (std::nothrow) fv_stats();
    if (!st) return fail(FV_ENOMEM, "host allocation failed");
    st->s = s;
    st->max_h = max_h;
    st->nq = s->nf;
    st->count = 0;
    // samples per pass: with structure functions, a chunk at a time (their partial sums); lags
    // beyond the staged kernels' reach also stage the chunk's quantities in qbuf. Without,
    // the whole batch goes through one Welford launch
    const int64_t state_bytes = (int64_t)sizeof(double) * st->nq * s->cells;
    st->chunk = max_h > 0 ? (int32_t)std::max<int64_t>(1, std::min<int64_t>(256, (512ll << 20) / state_bytes))
                          : (1 << 30);
    const size_t field = sizeof(double) * st->nq * s->cells;
    const size_t lags = sizeof(double) * st->nq * std::max(max_h, 1);
    const int32_t n32[3] = {(int32_t)s->grid.n[0], (int32_t)s->grid.n[1], (int32_t)s->grid.n[2]};
    const int nblk = max_h > 0 ? sf_blocks_per_field(s->grid.dim, n32, max_h) : 0;
    bool ok = hipMalloc((void**)&st->mean, field) == hipSuccess &&
              hipMalloc((void**)&st->m2, field) == hipSuccess &&
              hipMalloc((void**)&st->s2mean, lags) == hipSuccess &&
              hipMalloc((void**)&st->s2m2, lags) == hipSuccess;
    if (ok && max_h > 0)
        ok = (sf_staged(max_h) || hipMalloc((void**)&st->qbuf, field * st->chunk) == hipSuccess) &&
             hipMalloc((void**)&st->partial,
                       sizeof(double) * st->chunk * st->nq * max_h * (nblk + 1)) == hipSuccess;
    if (!ok) {
        fv_stats_destroy(st);
        return fail(FV_ENOMEM, "statistics allocation failed");
    }
    fv_status e = fv_stats_reset(st);
    if (e) {
        fv_stats_destroy(st);
        return e;
    }
    *out = st;
    return FV_OK;
}

extern "C" fv_status fv_stats_reset(fv_stats* st)
{
    if (!st) return fail(FV_EINVAL, "stats is NULL");
    hipStream_t str = st->s->stream;
    const int64_t field = (int64_t)st->nq * st->s->cells;
    const int64_t lags = (int64_t)st->nq * std::max(st->max_h, 1);
    launch_fill_zero(st->mean, field, str);
    launch_fill_zero(st->m2, field, str);
    launch_fill_zero(st->s2mean, lags, str);
    launch_fill_zero(st->s2m2, lags, str);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(str));
    st->count = 0;
    return FV_OK;
}

extern "C" fv_status fv_stats_accumulate(fv_stats* st, const double* state, int64_t batch)
{
    if (!st || !state) return fail(FV_EINVAL, "NULL argument");
    if (batch < 1) return fail(FV_EINVAL, "batch must be >= 1");
    fv_solver* s = const_cast<fv_solver*>(st->s);
    HIP_TRY(hipSetDevice(s->device));
    fv_status e = stream_enter(s);
    if (e) return e;
    hipStream_t str = s->stream;
    const int qkind = quantity_kind(s);
    const int64_t per = (int64_t)s->nf * s->cells;
    int32_t n32[3] = {(int32_t)s->grid.n[0], (int32_t)s->grid.n[1], (int32_t)s->grid.n[2]};
    const int nblk = st->max_h > 0 ? sf_blocks_per_field(s->grid.dim, n32, st->max_h) : 0;
    const double denom = (double)s->grid.dim * (double)s->cells;
    for (int64_t b0 = 0; b0 < batch; b0 += st->chunk) {
        const int32_t nb = (int32_t)std::min<int64_t>(st->chunk, batch - b0);
        const double* chunk = state + b0 * per;
        // the staged structure-function kernels form the quantities from the state themselves
        const bool staged = st->max_h > 0 && sf_staged(st->max_h);
        launch_welford(s->nf, qkind, chunk, s->cells, nb, st->count, st->mean, st->m2,
                       (st->max_h > 0 && !staged) ? st->qbuf : nullptr, str);
        if (st->max_h > 0) {
            if (staged)
                launch_sf_partial(chunk, s->grid.dim, n32, st->nq, st->max_h, nb, qkind,
                                  st->partial, str);
            else
                launch_sf_partial(st->qbuf, s->grid.dim, n32, st->nq, st->max_h, nb, -1,
                                  st->partial, str);
            // the per-sample values follow the partials in the same allocation
            double* xs = st->partial + (size_t)st->chunk * st->nq * st->max_h * nblk;
            launch_sf_welford(st->partial, st->nq, st->max_h, nblk, nb, st->count, denom, xs,
                              st->s2mean, st->s2m2, str);
        }
        HIP_TRY(hipGetLastError());
        st->count += nb;
    }
    return stream_leave(s);
}

static bool refinement_ratio(const fv_solver* f, const fv_solver* c, int32_t r[3])
{
    if (f->grid.dim != c->grid.dim || f->nf != c->nf || f->eq.kind != c->eq.kind) return false;
    for (int k = 0; k < 3; ++k) {
        if (c->grid.n[k] < 1 || f->grid.n[k] % c->grid.n[k] != 0) return false;
        r[k] = (int32_t)(f->grid.n[k] / c->grid.n[k]);
    }
    return true;
}

extern "C" fv_status fv_stats_accumulate_diff(fv_stats* st, const double* fine,
                                              const fv_solver* coarse, const double* coarse_state,
                                              int64_t batch)
{
    if (!st || !fine || !coarse || !coarse_state) return fail(FV_EINVAL, "NULL argument");
    if (batch < 1) return fail(FV_EINVAL, "batch must be >= 1");
    if (st->max_h != 0) return fail(FV_ENOTSUP, "level differences take no structure functions (max_h = 0)");
    fv_solver* s = const_cast<fv_solver*>(st->s);
    DiffGeom geo{};
    if (!refinement_ratio(s, coarse, geo.r))
        return fail(FV_EINVAL, "coarse grid must divide the fine grid on every axis, same equation");
    for (int k = 0; k < 3; ++k) {
        geo.nf[k] = (int32_t)s->grid.n[k];
        geo.nc[k] = (int32_t)coarse->grid.n[k];
    }
    HIP_TRY(hipSetDevice(s->device));
    fv_status e = stream_enter(s);
    if (e) return e;
    const int qkind = quantity_kind(s);
    const int64_t per_f = (int64_t)s->nf * s->cells, per_c = (int64_t)coarse->nf * coarse->cells;
    for (int64_t b0 = 0; b0 < batch; b0 += 1024) {
        const int32_t nb = (int32_t)std::min<int64_t>(1024, batch - b0);
        launch_welford_diff(s->nf, qkind, fine + b0 * per_f, coarse_state + b0 * per_c, geo, nb,
                            st->count, st->mean, st->m2, s->stream);
        HIP_TRY(hipGetLastError());
        st->count += nb;
    }
    return stream_leave(s);
}

extern "C" fv_status fv_mlmc_combine(int32_t nlevels, const fv_stats* const* levels, double* out)
{
    if (nlevels < 1 || nlevels > kMaxLevels) return fail(FV_EINVAL, "nlevels must be in [1, 8]");
    if (!levels || !out) return fail(FV_EINVAL, "NULL argument");
    const fv_stats* fin = levels[nlevels - 1];
    if (!fin) return fail(FV_EINVAL, "NULL level");
    const fv_solver* sf = fin->s;
    CombineArgs a{};
    a.nlevels = nlevels;
    a.nq = fin->nq;
    for (int k = 0; k < 3; ++k) a.nfine[k] = (int32_t)sf->grid.n[k];
    for (int l = 0; l < nlevels; ++l) {
        const fv_stats* lv = levels[l];
        if (!lv) return fail(FV_EINVAL, "NULL level");
        if (lv->count < 1) return fail(FV_EINVAL, "a level has no samples");
        if (!refinement_ratio(sf, lv->s, a.r[l])) return fail(FV_EINVAL, "levels must refine the finest grid");
        a.mean[l] = lv->mean;
        for (int k = 0; k < 3; ++k) a.n[l][k] = (int32_t)lv->s->grid.n[k];
    }
    fv_solver* s = const_cast<fv_solver*>(sf);
    HIP_TRY(hipSetDevice(s->device));
    for (int l = 0; l < nlevels; ++l) HIP_TRY(hipStreamSynchronize(levels[l]->s->stream));
    launch_mlmc_combine(a, out, s->stream);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s->stream));
    return FV_OK;
}

extern "C" fv_status fv_stats_read(const fv_stats* st, double* mean, double* var, double* s2_mean,
                                   double* s2_var, int64_t* count)
{
    if (!st) return fail(FV_EINVAL, "stats is NULL");
    fv_solver* s = const_cast<fv_solver*>(st->s);
    hipStream_t str = s->stream;
    const int64_t field = (int64_t)st->nq * s->cells;
    const int64_t lags = (int64_t)st->nq * st->max_h;
    if (count) *count = st->count;
    if (st->count < 1 && (var || s2_var)) return fail(FV_EINVAL, "no samples accumulated");
    if (mean) HIP_TRY(hipMemcpyAsync(mean, st->mean, sizeof(double) * field, hipMemcpyDeviceToDevice, str));
    if (var) launch_variance(st->m2, field, (double)st->count, var, str);
    if (lags > 0) {
        if (s2_mean) HIP_TRY(hipMemcpyAsync(s2_mean, st->s2mean, sizeof(double) * lags, hipMemcpyDeviceToDevice, str));
        if (s2_var) launch_variance(st->s2m2, lags, (double)st->count, s2_var, str);
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(str));
    return FV_OK;
}

extern "C" fv_status fv_stats_destroy(fv_stats* st)
{
    if (!st) return FV_OK;
    if (st->s && st->s->stream) hipStreamSynchronize(st->s->stream);
    hipFree(st->mean);
    hipFree(st->m2);
    hipFree(st->s2mean);
    hipFree(st->s2m2);
    hipFree(st->qbuf);
    hipFree(st->partial);
    delete st;
    return FV_OK;
}
