// fv_host.h -- host-side internals of libfv shared by its translation units (the solver
// object, error reporting, stream ordering). Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/fv.h"
#include "fv_common.h"
#include "fv_small.h"

extern thread_local std::string g_last_error;

inline fv_status fail(fv_status st, const std::string& msg)
{
    g_last_error = msg;
    return st;
}

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(FV_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));    \
    } while (0)

struct GraphCache {
    hipGraphExec_t exec = nullptr;
    std::vector<char> key;
};

struct fv_solver {
    fv_grid grid;
    fv_equation eq;
    int32_t flux, recon, integ;
    int32_t nf;
    int64_t cells;
    int32_t variant;
    const fvk::StageKernel* kern;
    // 1D grids small enough for one workgroup: the single-workgroup time loop, offered as
    // the variant after the tiled ones (use_small when it is the selected variant)
    const fvk::SmallKernel* small = nullptr;
    bool use_small = false;
    fvk::Phys ph;
    int device;
    hipStream_t user_stream = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    bool ws_owned = true;
    int32_t* host_count = nullptr;  // pinned
    GraphCache graph;
    // kernel timing (fv_profile_enable)
    bool profile = false;
    std::vector<hipEvent_t> prof_ev;
    double prof_stage_ms = 0.0;
    int64_t prof_stage_launches = 0;
    // small scratch for reductions (quantity of interest, line contraction)
    void* scratch = nullptr;
    size_t scratch_bytes = 0;
};

// Grow the solver's reduction scratch to at least `bytes` (synchronises the stream first).
inline fv_status ensure_scratch(fv_solver* s, size_t bytes)
{
    if (bytes <= s->scratch_bytes) return FV_OK;
    HIP_TRY(hipStreamSynchronize(s->stream));
    if (s->scratch) HIP_TRY(hipFree(s->scratch));
    s->scratch = nullptr;
    s->scratch_bytes = 0;
    if (hipMalloc(&s->scratch, bytes) != hipSuccess) return fail(FV_ENOMEM, "scratch allocation failed");
    s->scratch_bytes = bytes;
    return FV_OK;
}

// How the statistics turn a state into quantities: 0 the scalar itself; 1 Euler (rho,
// m_k (1/rho), E); 2 shallow water (h, hu_k (1/h)); 3 ideal MHD (rho, m_k (1/rho), E, B).
inline int quantity_kind(const fv_solver* s)
{
    return s->eq.kind == FV_EQ_EULER ? 1
           : (s->eq.kind == FV_EQ_SHALLOW_WATER ? 2 : (s->eq.kind == FV_EQ_MHD ? 3 : 0));
}

inline int n_stages(int integ) { return integ == FV_INT_FORWARD_EULER ? 1 : (integ == FV_INT_SSPRK2 ? 2 : 3); }

inline double stage_beta(int integ, int s)
{
    if (s == 0) return 1.0;
    if (integ == FV_INT_SSPRK2) return 0.5;
    return (s == 1) ? 0.25 : (2.0 / 3.0);
}

// Stage buffers: RK3 needs U^(1) and U^(2); RK2 and forward Euler need one.
inline int n_stage_buffers(int integ) { return integ == FV_INT_SSPRK3 ? 2 : 1; }

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

inline void drop_graph(fv_solver* s)
{
    if (s->graph.exec) hipGraphExecDestroy(s->graph.exec);
    s->graph.exec = nullptr;
    s->graph.key.clear();
}

// Order the private stream after the caller's stream, and the caller's after ours.
inline fv_status stream_enter(fv_solver* s)
{
    HIP_TRY(hipEventRecord(s->ev, s->user_stream));
    HIP_TRY(hipStreamWaitEvent(s->stream, s->ev, 0));
    return FV_OK;
}

inline fv_status stream_leave(fv_solver* s)
{
    HIP_TRY(hipEventRecord(s->ev, s->stream));
    HIP_TRY(hipStreamWaitEvent(s->user_stream, s->ev, 0));
    return FV_OK;
}
