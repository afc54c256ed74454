// fv_decomp.hip -- split-buffer domain decomposition of one grid on one GPU: the halo
// exchange of a multi-GPU run (Section 2.1, last paragraph; Section 3.1: splits along x, along
// y, and along both), emulated with device-to-device copies so that its schedule can be built
// and checked on one device.
//
// The grid is cut into parts[0] x parts[1] x parts[2] equal subdomains. Each subdomain has its
// own state arrays (U^n and the Runge--Kutta stage states) with G ghost layers stored on the
// split axes; every stage exchanges them:
//   pack    -- the G owned layers next to each face of every subdomain are gathered into a
//              contiguous send buffer, one message per (subdomain, split axis, side)
//              ("compactification": a strided face becomes one contiguous transfer);
//   copy    -- every message is copied device-to-device into the receive buffer on a second
//              stream (on several GPUs: a peer copy or an RCCL send/receive per neighbour);
//   unpack  -- the receive buffer is scattered into the ghost layers of the neighbour.
// With overlap, the stage kernel first updates the interior tiles (those whose haloed tile
// reads owned cells only) while the copies run, then waits for the copies' event, unpacks and
// updates the boundary shell. The per-cell arithmetic is that of the whole grid, and the
// maximum wave speed is merged over all subdomains exactly, so results are bit for bit those
// of the unsplit run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "fv_control.h"
#include "fv_host.h"
#include "fv_stage.h"

using namespace fvk;

namespace fvk {

constexpr int kMaxSub = 8;              // subdomains per decomposition (one launch's groups)
constexpr int kMaxMsg = kMaxSub * 6;    // messages per stage: (subdomain, axis, side)

// Halo-layout stage kernels: the tile shapes of the whole-grid defaults.
struct HaloEntry {
    int dim, eq, recon, flux;
    StageKernel k;
};

static const HaloEntry kHalo[] = {
    {2, EQ_EULER, REC_WENO3, FLUX_HLLC, make_stage_kernel<2, EQ_EULER, REC_WENO3, FLUX_HLLC, 16, 15, 1, 256, 2, 1>()},
    {2, EQ_EULER, REC_MUSCL, FLUX_HLL, make_stage_kernel<2, EQ_EULER, REC_MUSCL, FLUX_HLL, 16, 15, 1, 256, 2, 1>()},
    {2, EQ_EULER, REC_MUSCL, FLUX_RUSANOV, make_stage_kernel<2, EQ_EULER, REC_MUSCL, FLUX_RUSANOV, 16, 15, 1, 256, 2, 1>()},
    {3, EQ_EULER, REC_WENO3, FLUX_HLLC, make_stage_kernel<3, EQ_EULER, REC_WENO3, FLUX_HLLC, 8, 8, 4, 256, 1, 1>()},
};

static const StageKernel* find_halo_kernel(int dim, int eq, int recon, int flux)
{
    for (const HaloEntry& e : kHalo)
        if (e.dim == dim && e.eq == eq && e.recon == recon && e.flux == flux) return &e.k;
    return nullptr;
}

// One halo message: the G owned layers of subdomain src next to its `side` face along `axis`,
// for every sample and field, bound for the ghost layers of subdomain dst.
struct HaloMsg {
    int32_t src, dst, axis, side;   // side 0: low face (to dst's high ghosts), 1: high face
    int32_t e[3];                   // slab extent per axis (G along axis)
    int32_t pad;
    int64_t cells;                  // e[0] e[1] e[2]
    int64_t off;                    // first double in the send / receive buffers
};

struct SubPtrs {
    double* p[kMaxSub];
};

struct DecompGeom {
    int32_t nloc[3];   // owned cells per axis
    int32_t pn[3];     // array extent per axis
    int32_t off[3];    // offset of owned cell 0 per axis
    int32_t parts[3];
    int32_t nf;
    int32_t nsub;
    int32_t batch;
    int32_t g;         // ghost layers
    int32_t nmsg;
    int32_t pad;
    int64_t pcells;    // cells of one subdomain array (per field)
    int64_t n[3];      // the whole grid
};

// Whole grid <-> subdomain arrays (owned cells). dir 0: scatter, 1: gather.
__global__ void decomp_copy_kernel(const DecompGeom geo, const double* __restrict__ whole_in,
                                   double* __restrict__ whole_out, SubPtrs sub, int dir)
{
    const int64_t cells = geo.n[0] * geo.n[1] * geo.n[2];
    const int64_t total = cells * geo.nf * geo.batch;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = i % cells;
        const int64_t bq = i / cells;   // sample * nf + field
        const int64_t x = c % geo.n[0], y = (c / geo.n[0]) % geo.n[1], z = c / (geo.n[0] * geo.n[1]);
        const int32_t sx = (int32_t)(x / geo.nloc[0]), sy = (int32_t)(y / geo.nloc[1]),
                      sz = (int32_t)(z / geo.nloc[2]);
        const int32_t s = (sz * geo.parts[1] + sy) * geo.parts[0] + sx;
        const int64_t lx = x - (int64_t)sx * geo.nloc[0] + geo.off[0];
        const int64_t ly = y - (int64_t)sy * geo.nloc[1] + geo.off[1];
        const int64_t lz = z - (int64_t)sz * geo.nloc[2] + geo.off[2];
        const int64_t a = bq * geo.pcells + (lz * geo.pn[1] + ly) * geo.pn[0] + lx;
        if (dir == 0) sub.p[s][a] = whole_in[i];
        else whole_out[i] = sub.p[s][a];
    }
}

// Slab cell c of message m (x fastest within the slab) -> its array index in the sending
// subdomain (from = true) or in the receiving one's ghost layers, for sample-field bq.
__device__ __forceinline__ int64_t msg_array_index(const DecompGeom& geo, const HaloMsg& m,
                                                   int64_t bq, uint32_t c, bool from)
{
    const uint32_t e0 = (uint32_t)m.e[0], e1 = (uint32_t)m.e[1];
    int32_t l[3];
    const uint32_t t = c / e0;
    l[0] = (int32_t)(c - t * e0);
    l[1] = (int32_t)(t % e1);
    l[2] = (int32_t)(t / e1);
    const int a = m.axis;
    if (from) l[a] = (m.side == 0) ? l[a] : geo.nloc[a] - geo.g + l[a];
    else l[a] = (m.side == 0) ? geo.nloc[a] + l[a] : l[a] - geo.g;
    return bq * geo.pcells + ((int64_t)(l[2] + geo.off[2]) * geo.pn[1] + (l[1] + geo.off[1])) * geo.pn[0] +
           (l[0] + geo.off[0]);
}

// pack (dir 0): subdomain arrays -> send buffer; unpack (dir 1): receive buffer -> ghosts.
// Grid: (blocks over a slab's cells, message, sample * field); buffer layout
// [message][sample][field][slab cell].
__global__ void halo_kernel(const DecompGeom geo, const HaloMsg* __restrict__ msg, SubPtrs arr,
                            double* __restrict__ buf, int dir)
{
    const HaloMsg& m = msg[blockIdx.y];
    const int64_t bq = blockIdx.z;
    double* B = buf + m.off + bq * m.cells;
    for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < (uint32_t)m.cells;
         c += gridDim.x * blockDim.x) {
        if (dir == 0) B[c] = arr.p[m.src][msg_array_index(geo, m, bq, c, true)];
        else arr.p[m.dst][msg_array_index(geo, m, bq, c, false)] = B[c];
    }
}

}  // namespace fvk

struct fv_decomp {
    fv_solver* s = nullptr;
    const StageKernel* hk = nullptr;
    DecompGeom geo{};
    int32_t hmask = 0;
    int nst = 0;
    // per subdomain: U^n, stage states
    double* U[kMaxSub] = {};
    double* W[2][kMaxSub] = {};
    double* send = nullptr;
    double* recv = nullptr;
    HaloMsg* msg_dev = nullptr;
    std::vector<HaloMsg> msgs;
    // one copy per (sending, receiving) subdomain pair: consecutive messages between the same
    // pair are contiguous in the buffers (offset, doubles)
    std::vector<std::pair<int64_t, int64_t>> transfers;
    int64_t msg_doubles = 0;        // doubles of all messages of one stage
    // interior box and shell boxes of every subdomain's tiles (same for all subdomains)
    int32_t tiles[3] = {1, 1, 1};
    int32_t ilo[3] = {0, 0, 0}, ihi[3] = {1, 1, 1};
    std::vector<std::pair<std::array<int32_t, 3>, std::array<int32_t, 3>>> shell;   // (lo, count)
    // control words
    double* dt = nullptr;
    unsigned long long* mbits = nullptr;
    int32_t* running = nullptr;
    int32_t* active = nullptr;
    int32_t* bad = nullptr;
    int64_t* steps = nullptr;
    int32_t* err = nullptr;
    int32_t* count = nullptr;       // [1 + kMaxGroups] running counts, then the first error
    int32_t* host = nullptr;        // pinned
    hipStream_t copy = nullptr;
    hipEvent_t ev_pack = nullptr, ev_copy = nullptr;   // pack done; copies (+ shell) done
    // captured chunk of steps (key: the run's settings and pointers)
    hipGraphExec_t exec = nullptr;
    std::vector<char> key;
    // timing
    bool profile = false;
    std::vector<hipEvent_t> prof;   // per step: compute start/end; per stage: copy start/end
    double step_ms = 0.0, copy_ms = 0.0;
    int64_t prof_steps = 0;
};

static void decomp_free(fv_decomp* d)
{
    for (int i = 0; i < kMaxSub; ++i) {
        hipFree(d->U[i]);
        hipFree(d->W[0][i]);
        hipFree(d->W[1][i]);
    }
    hipFree(d->send);
    hipFree(d->recv);
    hipFree(d->msg_dev);
    hipFree(d->dt);
    hipFree(d->mbits);
    hipFree(d->running);
    hipFree(d->active);
    hipFree(d->bad);
    hipFree(d->steps);
    hipFree(d->err);
    hipFree(d->count);
    if (d->host) hipHostFree(d->host);
    for (hipEvent_t e : d->prof) hipEventDestroy(e);
    if (d->exec) hipGraphExecDestroy(d->exec);
    if (d->ev_pack) hipEventDestroy(d->ev_pack);
    if (d->ev_copy) hipEventDestroy(d->ev_copy);
    if (d->copy) hipStreamDestroy(d->copy);
    delete d;
}

extern "C" fv_status fv_decomp_create(fv_solver* s, const int32_t* parts, int64_t batch,
                                      fv_decomp** out)
{
    if (!s || !parts || !out) return fail(FV_EINVAL, "NULL argument");
    *out = nullptr;
    if (batch < 1 || batch > 8192) return fail(FV_EINVAL, "batch must be in [1, 8192]");
    const int dim = s->grid.dim;
    int nsub = 1;
    for (int k = 0; k < 3; ++k) {
        if (parts[k] < 1) return fail(FV_EINVAL, "parts must be >= 1");
        if (k >= dim && parts[k] != 1) return fail(FV_EINVAL, "parts must be 1 beyond the grid's dimension");
        nsub *= parts[k];
    }
    if (nsub > kMaxSub) return fail(FV_ENOTSUP, "at most 8 subdomains");
    if (s->integ == FV_INT_FORWARD_EULER)
        return fail(FV_ENOTSUP, "split runs take the SSP Runge--Kutta steppers (2 or 3 stages)");
    const StageKernel* hk = find_halo_kernel(dim, s->eq.kind, s->recon, s->flux);
    if (!hk)
        return fail(FV_ENOTSUP, "split runs cover the Euler equations with WENO3 + HLLC (2D, 3D), "
                                "MUSCL + HLL and MUSCL + Rusanov (2D)");
    const int G = (s->recon == FV_RECON_FIRST_ORDER) ? 1 : 2;
    DecompGeom geo{};
    int32_t hmask = 0;
    int64_t pcells = 1;
    for (int k = 0; k < 3; ++k) {
        geo.n[k] = s->grid.n[k];
        geo.parts[k] = parts[k];
        if (s->grid.n[k] % parts[k] != 0) return fail(FV_EINVAL, "parts must divide the grid on every axis");
        geo.nloc[k] = (int32_t)(s->grid.n[k] / parts[k]);
        const bool split = parts[k] > 1;
        if (split) {
            if (s->grid.bc[k] != FV_BC_PERIODIC) return fail(FV_ENOTSUP, "split axes must be periodic");
            if (geo.nloc[k] < 2 * G) return fail(FV_EINVAL, "subdomains need at least 2 ghost widths of cells per split axis");
            hmask |= 1 << k;
        }
        geo.off[k] = split ? G : 0;
        geo.pn[k] = geo.nloc[k] + 2 * geo.off[k];
        pcells *= geo.pn[k];
    }
    if (pcells > INT32_MAX) return fail(FV_EINVAL, "subdomain array too large");
    geo.nf = s->nf;
    geo.nsub = nsub;
    geo.batch = (int32_t)batch;
    geo.g = G;
    geo.pcells = pcells;

    fv_decomp* d = new (std::nothrow) fv_decomp();
    if (!d) return fail(FV_ENOMEM, "host allocation failed");
    d->s = s;
    d->hk = hk;
    d->hmask = hmask;
    d->nst = n_stages(s->integ);

    // messages: (subdomain, split axis, side), in that order
    int64_t off = 0;
    for (int sub = 0; sub < nsub; ++sub) {
        const int sx = sub % parts[0], sy = (sub / parts[0]) % parts[1], sz = sub / (parts[0] * parts[1]);
        const int sc[3] = {sx, sy, sz};
        for (int a = 0; a < 3; ++a) {
            if (!(hmask & (1 << a))) continue;
            for (int side = 0; side < 2; ++side) {
                HaloMsg m{};
                m.src = sub;
                int nc[3] = {sc[0], sc[1], sc[2]};
                nc[a] = (sc[a] + (side == 0 ? parts[a] - 1 : 1)) % parts[a];
                m.dst = (nc[2] * parts[1] + nc[1]) * parts[0] + nc[0];
                m.axis = a;
                m.side = side;
                for (int k = 0; k < 3; ++k) m.e[k] = (k == a) ? G : geo.nloc[k];
                m.cells = (int64_t)m.e[0] * m.e[1] * m.e[2];
                m.off = off;
                off += m.cells * geo.nf * batch;
                d->msgs.push_back(m);
            }
        }
    }
    geo.nmsg = (int32_t)d->msgs.size();
    d->msg_doubles = off;
    for (size_t i = 0; i < d->msgs.size(); ++i) {
        const HaloMsg& m = d->msgs[i];
        const int64_t nd = m.cells * geo.nf * batch;
        if (i > 0 && d->msgs[i - 1].src == m.src && d->msgs[i - 1].dst == m.dst)
            d->transfers.back().second += nd;
        else
            d->transfers.push_back({m.off, nd});
    }
    d->geo = geo;

    // tiles of a subdomain: interior along a split axis = tiles whose haloed extent stays in
    // the owned cells, [1, (nloc - G) / B)
    const int32_t B[3] = {hk->bx, hk->by, hk->bz};
    for (int k = 0; k < 3; ++k) {
        d->tiles[k] = (geo.nloc[k] + B[k] - 1) / B[k];
        if (hmask & (1 << k)) {
            d->ilo[k] = 1;
            d->ihi[k] = std::max(1, (geo.nloc[k] - G) / B[k]);
        } else {
            d->ilo[k] = 0;
            d->ihi[k] = d->tiles[k];
        }
    }
    {   // boundary shell: slabs along x, then y within the interior x range, then z
        int32_t lo[3] = {0, 0, 0}, hi[3] = {d->tiles[0], d->tiles[1], d->tiles[2]};
        for (int k = 0; k < 3; ++k) {
            if (!(hmask & (1 << k))) continue;
            for (int side = 0; side < 2; ++side) {
                std::array<int32_t, 3> blo{lo[0], lo[1], lo[2]}, bcnt{};
                for (int j = 0; j < 3; ++j) bcnt[j] = hi[j] - lo[j];
                if (side == 0) { blo[k] = 0; bcnt[k] = d->ilo[k]; }
                else { blo[k] = d->ihi[k]; bcnt[k] = d->tiles[k] - d->ihi[k]; }
                if (bcnt[0] > 0 && bcnt[1] > 0 && bcnt[2] > 0) d->shell.push_back({blo, bcnt});
            }
            lo[k] = d->ilo[k];
            hi[k] = d->ihi[k];
        }
    }

    const size_t sb = sizeof(double) * (size_t)pcells * geo.nf * batch;
    bool ok = hipSetDevice(s->device) == hipSuccess;
    for (int i = 0; ok && i < nsub; ++i) {
        ok = hipMalloc((void**)&d->U[i], sb) == hipSuccess && hipMemset(d->U[i], 0, sb) == hipSuccess;
        for (int w = 0; ok && w < d->nst - 1; ++w)
            ok = hipMalloc((void**)&d->W[w][i], sb) == hipSuccess && hipMemset(d->W[w][i], 0, sb) == hipSuccess;
    }
    const size_t mb = sizeof(double) * (size_t)std::max<int64_t>(1, off);
    ok = ok && hipMalloc((void**)&d->send, mb) == hipSuccess && hipMalloc((void**)&d->recv, mb) == hipSuccess &&
         hipMalloc((void**)&d->msg_dev, sizeof(HaloMsg) * std::max<size_t>(1, d->msgs.size())) == hipSuccess &&
         hipMalloc((void**)&d->dt, sizeof(double) * batch) == hipSuccess &&
         hipMalloc((void**)&d->mbits, sizeof(unsigned long long) * kSpeedSlots * speed_pitch(batch)) == hipSuccess &&
         hipMalloc((void**)&d->running, sizeof(int32_t) * batch) == hipSuccess &&
         hipMalloc((void**)&d->active, sizeof(int32_t) * batch) == hipSuccess &&
         hipMalloc((void**)&d->bad, sizeof(int32_t) * batch) == hipSuccess &&
         hipMalloc((void**)&d->steps, sizeof(int64_t) * batch) == hipSuccess &&
         hipMalloc((void**)&d->err, sizeof(int32_t) * batch) == hipSuccess &&
         hipMalloc((void**)&d->count, sizeof(int32_t) * (2 + kMaxGroups)) == hipSuccess &&
         hipHostMalloc((void**)&d->host, sizeof(int32_t) * (2 + kMaxGroups), hipHostMallocDefault) == hipSuccess &&
         hipStreamCreateWithFlags(&d->copy, hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&d->ev_pack, hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&d->ev_copy, hipEventDisableTiming) == hipSuccess;
    if (ok && !d->msgs.empty())
        ok = hipMemcpy(d->msg_dev, d->msgs.data(), sizeof(HaloMsg) * d->msgs.size(),
                       hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) {
        decomp_free(d);
        return fail(FV_ENOMEM, "decomposition allocation failed");
    }
    *out = d;
    return FV_OK;
}

extern "C" fv_status fv_decomp_destroy(fv_decomp* d)
{
    if (!d) return FV_OK;
    if (d->s && d->s->stream) hipStreamSynchronize(d->s->stream);
    if (d->copy) hipStreamSynchronize(d->copy);
    decomp_free(d);
    return FV_OK;
}

static SubPtrs ptrs_of(double* const* a, int n)
{
    SubPtrs p{};
    for (int i = 0; i < n; ++i) p.p[i] = a[i];
    return p;
}

static fv_status decomp_copy(fv_decomp* d, const double* in, double* out, int dir)
{
    fv_solver* s = d->s;
    HIP_TRY(hipSetDevice(s->device));
    fv_status e = stream_enter(s);
    if (e) return e;
    hipLaunchKernelGGL(decomp_copy_kernel, dim3(2048), dim3(256), 0, s->stream, d->geo, in, out,
                       ptrs_of(d->U, d->geo.nsub), dir);
    HIP_TRY(hipGetLastError());
    return stream_leave(s);
}

extern "C" fv_status fv_decomp_scatter(fv_decomp* d, const double* state)
{
    if (!d || !state) return fail(FV_EINVAL, "NULL argument");
    return decomp_copy(d, state, nullptr, 0);
}

extern "C" fv_status fv_decomp_gather(fv_decomp* d, double* state)
{
    if (!d || !state) return fail(FV_EINVAL, "NULL argument");
    return decomp_copy(d, nullptr, state, 1);
}

// Group of subdomain `sub` for a launch over the tile box (lo, cnt).
static Group decomp_group(const fv_decomp* d, int sub, const double* src, const double* un,
                          double* dst, const int32_t* lo, const int32_t* cnt)
{
    Group g{};
    g.src = src;
    g.un = un;
    g.dst = dst;
    g.dt = d->dt;
    g.active = d->active;
    g.mbits = d->mbits;
    g.bad = d->bad;
    g.cells = d->geo.pcells;
    g.ntiles = 1;
    for (int k = 0; k < 3; ++k) {
        g.n[k] = d->geo.nloc[k];
        g.tiles[k] = d->tiles[k];
        g.pn[k] = d->geo.pn[k];
        g.off[k] = d->geo.off[k];
        g.tlo[k] = lo[k];
        g.tcnt[k] = cnt[k];
        g.ntiles *= cnt[k];
    }
    g.hmask = d->hmask;
    g.batch = d->geo.batch;
    g.ph = d->s->ph;
    (void)sub;
    return g;
}

// One stage launch over a list of (subdomain, box) pieces, in launches of <= kMaxGroups groups.
struct Piece {
    int sub;
    int32_t lo[3], cnt[3];
};

static void stage_launches(fv_decomp* d, const std::vector<Piece>& pieces, double* const* src,
                           double* const* un, double* const* dst, int stage, hipStream_t str)
{
    const fv_solver* s = d->s;
    for (size_t p0 = 0; p0 < pieces.size(); p0 += kMaxGroups) {
        StageArgs a{};
        int64_t blocks = 0;
        for (size_t i = p0; i < std::min(pieces.size(), p0 + kMaxGroups); ++i) {
            const Piece& pc = pieces[i];
            Group g = decomp_group(d, pc.sub, src[pc.sub], un[pc.sub], dst[pc.sub], pc.lo, pc.cnt);
            g.block0 = blocks;
            blocks += (int64_t)g.ntiles * g.batch;
            a.g[a.ngroups++] = g;
        }
        if (blocks == 0) continue;
        for (int k = 0; k < 3; ++k) a.bc[k] = s->grid.bc[k];
        a.beta = stage_beta(s->integ, stage);
        a.use_un = stage > 0;
        a.last = (stage == d->nst - 1);
        a.nblocks = blocks;
        d->hk->stage(a, str);
    }
}

// Grid of the pack / unpack kernel: enough blocks for the largest slab (at most 1024),
// every message, every sample-field.
static dim3 halo_grid(const fv_decomp* d)
{
    int64_t most = 1;
    for (const HaloMsg& m : d->msgs) most = std::max<int64_t>(most, m.cells);
    return dim3((unsigned)std::min<int64_t>(1024, (most + 255) / 256), (unsigned)d->msgs.size(),
                (unsigned)(d->geo.nf * d->geo.batch));
}

static void exchange_start(fv_decomp* d, double* const* arr, hipEvent_t* cev, bool dma)
{
    const fv_solver* s = d->s;
    const int64_t total = d->msg_doubles;
    if (total == 0) return;
    hipLaunchKernelGGL(halo_kernel, halo_grid(d), dim3(256), 0, s->stream, d->geo, d->msg_dev,
                       ptrs_of(arr, d->geo.nsub), d->send, 0);
    hipEventRecord(d->ev_pack, s->stream);
    hipStreamWaitEvent(d->copy, d->ev_pack, 0);
    if (cev) hipEventRecord(cev[0], d->copy);
    for (const auto& tr : d->transfers)
        hipMemcpyAsync(d->recv + tr.first, d->send + tr.first, sizeof(double) * (size_t)tr.second,
                       dma ? hipMemcpyDeviceToDeviceNoCU : hipMemcpyDeviceToDevice, d->copy);
    if (cev) hipEventRecord(cev[1], d->copy);
}

// Unpack into the ghost layers, on stream str (after the copies when str is the copy stream;
// the solver's stream waits for the copies first otherwise).
static void exchange_finish(fv_decomp* d, double* const* arr, hipStream_t str)
{
    const fv_solver* s = d->s;
    const int64_t total = d->msg_doubles;
    if (total == 0) return;
    if (str == s->stream) {
        hipEventRecord(d->ev_copy, d->copy);
        hipStreamWaitEvent(s->stream, d->ev_copy, 0);
    }
    hipLaunchKernelGGL(halo_kernel, halo_grid(d), dim3(256), 0, str, d->geo, d->msg_dev,
                       ptrs_of(arr, d->geo.nsub), d->recv, 1);
}

static CtrlArgs decomp_ctrl(fv_decomp* d, double* t, int64_t* steps, int32_t* err, double t_end,
                            double cfl, int64_t max_steps)
{
    CtrlArgs c{};
    c.ngroups = 1;
    CtrlGroup& g = c.g[0];
    g.t = t;
    g.dt = d->dt;
    g.running = d->running;
    g.active = d->active;
    g.mbits = d->mbits;
    g.bad = d->bad;
    g.steps = steps ? steps : d->steps;
    g.err = err ? err : d->err;
    g.batch = d->geo.batch;
    c.fixed = 0;
    c.limit_is_error = 0;
    c.t_end = t_end;
    c.cfl = cfl;
    c.max_steps = max_steps;
    c.n_running = d->count;
    return c;
}

extern "C" fv_status fv_decomp_advance(fv_decomp* d, double* t, double t_end, double cfl,
                                       int64_t nsteps, int64_t* steps, int32_t* err,
                                       int32_t mode)
{
    if (!d || !t) return fail(FV_EINVAL, "NULL argument");
    if (mode < 0 || mode > 3) return fail(FV_EINVAL, "mode must be 0..3 (overlap | DMA copies)");
    if (!(cfl > 0.0) || cfl > 1.0) return fail(FV_EINVAL, "cfl must be in (0, 1]");
    if (!std::isfinite(t_end)) return fail(FV_EINVAL, "t_end must be finite");
    if (nsteps < 0) return fail(FV_EINVAL, "nsteps must be >= 0");
    fv_solver* s = d->s;
    HIP_TRY(hipSetDevice(s->device));
    fv_status e = stream_enter(s);
    if (e) return e;
    hipStream_t st = s->stream;
    const int P = d->geo.nsub;
    const CtrlArgs ctrl = decomp_ctrl(d, t, steps, err, t_end, cfl, nsteps);
    launch_ctrl_reset(ctrl, st);
    {   // wave speed of the initial state, over the owned cells of every subdomain
        SpeedArgs sp{};
        int64_t blocks = 0;
        const int32_t zero[3] = {0, 0, 0};
        for (int i = 0; i < P; ++i) {
            Group g = decomp_group(d, i, d->U[i], d->U[i], nullptr, zero, d->tiles);
            g.block0 = blocks;
            const int64_t owned = (int64_t)g.n[0] * g.n[1] * g.n[2];
            blocks += (owned + d->hk->cells_per_block - 1) / d->hk->cells_per_block * g.batch;
            sp.g[sp.ngroups++] = g;
        }
        sp.nblocks = blocks;
        d->hk->speed(sp, st);
    }
    launch_ctrl_begin(ctrl, st);
    HIP_TRY(hipGetLastError());

    // pieces: the whole subdomain, its interior box, its boundary shell
    std::vector<Piece> whole, inner, shell;
    for (int i = 0; i < P; ++i) {
        Piece w{i, {0, 0, 0}, {d->tiles[0], d->tiles[1], d->tiles[2]}};
        whole.push_back(w);
        Piece in{i, {d->ilo[0], d->ilo[1], d->ilo[2]},
                 {d->ihi[0] - d->ilo[0], d->ihi[1] - d->ilo[1], d->ihi[2] - d->ilo[2]}};
        if (in.cnt[0] > 0 && in.cnt[1] > 0 && in.cnt[2] > 0) inner.push_back(in);
        for (const auto& b : d->shell) {
            Piece sh{i, {b.first[0], b.first[1], b.first[2]}, {b.second[0], b.second[1], b.second[2]}};
            shell.push_back(sh);
        }
    }
    // inner + shell cover every tile once (an empty interior leaves everything in the shell)
    if (inner.empty()) shell = whole;

    const int S = d->nst;
    double* un[kMaxSub];
    double* w1[kMaxSub];
    double* w2[kMaxSub];
    for (int i = 0; i < P; ++i) {
        un[i] = d->U[i];
        w1[i] = d->W[0][i];
        w2[i] = d->W[1][i];
    }
    // sources and destinations per stage: RK3 U -> W1 -> W2 -> U, RK2 U -> W1 -> U
    double* const* srcs[3] = {un, w1, w2};
    double* const* dsts[3] = {w1, (S == 3) ? w2 : un, un};

    const size_t per_step_ev = 2 + 2 * (size_t)S;
    if (d->profile) {
        while (d->prof.size() < per_step_ev * (size_t)nsteps) {
            hipEvent_t ev;
            HIP_TRY(hipEventCreate(&ev));
            d->prof.push_back(ev);
        }
    }
    auto step = [&](hipEvent_t* ev) {
        if (ev) hipEventRecord(ev[0], st);
        for (int stg = 0; stg < S; ++stg) {
            double* const* src = srcs[stg];
            double* const* dst = dsts[stg];
            exchange_start(d, src, ev ? ev + 2 + 2 * stg : nullptr, (mode & 2) != 0);
            if ((mode & 1) && d->msg_doubles > 0) {
                // the interior on the solver's stream; the unpack and the boundary shell on the
                // copy stream right behind the copies, concurrent with the interior; the next
                // stage waits for both (the two tile sets are disjoint, the unpack writes only
                // ghost layers, which interior tiles do not read)
                stage_launches(d, inner, src, un, dst, stg, st);
                exchange_finish(d, src, d->copy);
                stage_launches(d, shell, src, un, dst, stg, d->copy);
                hipEventRecord(d->ev_copy, d->copy);
                hipStreamWaitEvent(st, d->ev_copy, 0);
            } else {
                exchange_finish(d, src, st);
                stage_launches(d, whole, src, un, dst, stg, st);
            }
        }
        launch_ctrl_begin(ctrl, st);
        if (ev) hipEventRecord(ev[1], st);
    };
    // Without timing, whole chunks of steps replay a graph captured over both streams (the
    // copy stream forks from and joins the solver's stream through the exchange events); the
    // remainder is enqueued directly. A finished sample's launches return at once.
    constexpr int64_t kChunk = 16;
    const char* ng = std::getenv("FV_NO_GRAPH");
    const bool graphs = !d->profile && !(ng && ng[0] && ng[0] != '0');
    int64_t n = 0;
    if (graphs && nsteps >= kChunk) {
        std::vector<char> key;
        auto push = [&](const void* p, size_t b) {
            const char* c = (const char*)p;
            key.insert(key.end(), c, c + b);
        };
        push(&t, sizeof t); push(&steps, sizeof steps); push(&err, sizeof err);
        push(&t_end, sizeof t_end); push(&cfl, sizeof cfl); push(&nsteps, sizeof nsteps);
        push(&mode, sizeof mode);
        if (!d->exec || d->key != key) {
            if (d->exec) HIP_TRY(hipGraphExecDestroy(d->exec));
            d->exec = nullptr;
            hipGraph_t gr = nullptr;
            HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            for (int64_t i = 0; i < kChunk; ++i) step(nullptr);
            const hipError_t ce = hipStreamEndCapture(st, &gr);
            if (ce != hipSuccess) return fail(FV_EDEVICE, std::string("graph capture: ") + hipGetErrorString(ce));
            const hipError_t ie = hipGraphInstantiate(&d->exec, gr, nullptr, nullptr, 0);
            hipGraphDestroy(gr);
            if (ie != hipSuccess) return fail(FV_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(ie));
            d->key = key;
        }
        for (; n + kChunk <= nsteps; n += kChunk) HIP_TRY(hipGraphLaunch(d->exec, st));
    }
    for (; n < nsteps; ++n) {
        step(d->profile ? &d->prof[per_step_ev * (size_t)n] : nullptr);
        HIP_TRY(hipGetLastError());
    }
    // the first failing sample
    launch_first_error(ctrl.g[0].err, d->geo.batch, d->count + kMaxGroups, st);
    HIP_TRY(hipMemcpyAsync(d->host, d->count + kMaxGroups, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    HIP_TRY(hipStreamSynchronize(d->copy));
    if (d->profile) {
        for (int64_t n = 0; n < nsteps; ++n) {
            hipEvent_t* ev = &d->prof[per_step_ev * (size_t)n];
            float ms = 0.0f;
            HIP_TRY(hipEventElapsedTime(&ms, ev[0], ev[1]));
            d->step_ms += ms;
            for (int stg = 0; stg < S && d->msg_doubles > 0; ++stg) {
                HIP_TRY(hipEventElapsedTime(&ms, ev[2 + 2 * stg], ev[3 + 2 * stg]));
                d->copy_ms += ms;
            }
        }
        d->prof_steps += nsteps;
    }
    e = stream_leave(s);
    if (e) return e;
    if (d->host[0] != 0) {
        g_last_error = "sample " + std::to_string(d->host[1]) + " failed with status " +
                       std::to_string(d->host[0]);
        return (fv_status)d->host[0];
    }
    return FV_OK;
}

extern "C" fv_status fv_decomp_profile_enable(fv_decomp* d, int32_t on)
{
    if (!d) return fail(FV_EINVAL, "decomposition is NULL");
    d->profile = on != 0;
    d->step_ms = d->copy_ms = 0.0;
    d->prof_steps = 0;
    return FV_OK;
}

extern "C" fv_status fv_decomp_profile_read(const fv_decomp* d, double* step_ms, double* copy_ms,
                                            int64_t* steps)
{
    if (!d) return fail(FV_EINVAL, "decomposition is NULL");
    if (step_ms) *step_ms = d->step_ms;
    if (copy_ms) *copy_ms = d->copy_ms;
    if (steps) *steps = d->prof_steps;
    return FV_OK;
}

extern "C" fv_status fv_decomp_info(const fv_decomp* d, int32_t* nsub, int32_t* messages,
                                    int64_t* halo_bytes, int32_t* interior_tiles,
                                    int32_t* shell_tiles)
{
    if (!d) return fail(FV_EINVAL, "decomposition is NULL");
    if (nsub) *nsub = d->geo.nsub;
    if (messages) *messages = (int32_t)d->msgs.size();
    if (halo_bytes) *halo_bytes = (int64_t)sizeof(double) * d->msg_doubles;
    int64_t inner = 1, all = 1;
    for (int k = 0; k < 3; ++k) {
        inner *= std::max(0, d->ihi[k] - d->ilo[k]);
        all *= d->tiles[k];
    }
    if (interior_tiles) *interior_tiles = (int32_t)inner;
    if (shell_tiles) *shell_tiles = (int32_t)(all - inner);
    return FV_OK;
}
