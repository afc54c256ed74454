// fv_control.hip -- per-sample step control kept on the device, so that a whole chunk of
// time steps can be enqueued (and captured in a HIP graph) without host round trips.
//
// Each sample b carries: time t[b], step size dt[b], step count steps[b], status err[b],
// running[b] (still evolving), active[b] (takes the current step), the maximum wave speed
// mbits[b] of its current state (bit pattern of a non-negative double, merged with an atomic
// max by the last Runge--Kutta stage) and bad[b] (a non-physical value was seen).
#include "fv_control.h"

namespace fvk {

__global__ void ctrl_reset_kernel(const CtrlArgs a)
{
    for (int gi = 0; gi < a.ngroups; ++gi) {
        const CtrlGroup& g = a.g[gi];
        const int64_t pitch = speed_pitch(g.batch);
        for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < g.batch; b += gridDim.x * blockDim.x) {
            g.running[b] = 1;
            g.active[b] = 1;
            for (int s = 0; s < kSpeedSlots; ++s) g.mbits[s * pitch + b] = 0ull;
            g.bad[b] = 0;
            g.steps[b] = 0;
            g.err[b] = ST_OK;
            g.dt[b] = 0.0;
        }
    }
}

// Decide, for every sample, whether and with which dt it takes the next step; count the
// samples still running into *n_running. Launched with one workgroup.
__global__ void __launch_bounds__(1024) ctrl_begin_kernel(const CtrlArgs a)
{
    __shared__ int count[kMaxGroups];
    if (threadIdx.x < kMaxGroups) count[threadIdx.x] = 0;
    __syncthreads();
    for (int gi = 0; gi < a.ngroups; ++gi) {
        const CtrlGroup& g = a.g[gi];
        const int64_t pitch = speed_pitch(g.batch);
        int mine = 0;
        for (int b = threadIdx.x; b < g.batch; b += blockDim.x) {
            if (!g.running[b]) { g.active[b] = 0; continue; }
            int stop = 0;
            int32_t e = ST_OK;
            // bit patterns of non-negative doubles order like the doubles
            unsigned long long mb = 0ull;
            for (int s = 0; s < kSpeedSlots; ++s) {
                const unsigned long long v = g.mbits[s * pitch + b];
                mb = v > mb ? v : mb;
            }
            const double M = __longlong_as_double((long long)mb);
            double dt = 0.0, tnew = 0.0;
            if (g.bad[b]) {
                e = ST_ENONPHYS;
                stop = 1;
            } else if (a.fixed) {
                if (g.steps[b] >= a.max_steps) {
                    stop = 1;
                } else if (a.fixed_dt * M > a.cfl_bound) {
                    e = ST_ECFL;
                    stop = 1;
                } else {
                    dt = a.fixed_dt;
                }
            } else {
                const double t = g.t[b];
                if (!(t < a.t_end)) {
                    stop = 1;
                } else if (g.steps[b] >= a.max_steps) {
                    if (a.limit_is_error) e = ST_EMAXSTEPS;
                    stop = 1;
                } else {
                    dt = (M == 0.0) ? (a.t_end - t) : (a.cfl / M);
                    bool last = false;
                    if (t + dt >= a.t_end) {
                        dt = a.t_end - t;
                        last = true;
                    }
                    tnew = last ? a.t_end : (t + dt);
                }
            }
            if (stop) {
                g.err[b] = e;
                g.running[b] = 0;
                g.active[b] = 0;
                continue;
            }
            g.dt[b] = dt;
            if (!a.fixed) g.t[b] = tnew;
            g.steps[b] = g.steps[b] + 1;
            g.active[b] = 1;
            for (int s = 0; s < kSpeedSlots; ++s) g.mbits[s * pitch + b] = 0ull;
            g.bad[b] = 0;
            mine += 1;
        }
        if (mine) atomicAdd(&count[gi], mine);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int total = 0;
        for (int gi = 0; gi < a.ngroups; ++gi) {
            total += count[gi];
            a.n_running[1 + gi] = count[gi];
        }
        a.n_running[0] = total;
    }
}

// Forward Euler has a single stage that cannot update in place (neighbours read the old
// state); it writes a stage buffer that this kernel copies back for the active samples.
__global__ void copy_back_kernel(const CopyArgs a)
{
    const int gi = blockIdx.y;
    if (gi >= a.ngroups) return;
    const CopyGroup& g = a.g[gi];
    const int64_t per = g.per_sample;
    const int64_t total = per * g.batch;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = i / per;
        if (g.active[b]) g.dst[i] = g.src[i];
    }
}

// The status of the first failing sample: out[0] = err[b] and out[1] = b for the smallest b
// with err[b] != 0, or out[0] = 0 and out[1] = -1 when every sample succeeded. One workgroup.
__global__ void __launch_bounds__(1024) first_error_kernel(const int32_t* __restrict__ err,
                                                           int32_t batch, int32_t* __restrict__ out)
{
    __shared__ int first;
    if (threadIdx.x == 0) first = INT32_MAX;
    __syncthreads();
    for (int b = threadIdx.x; b < batch; b += blockDim.x)
        if (err[b] != 0) {
            atomicMin(&first, b);
            break;
        }
    __syncthreads();
    if (threadIdx.x == 0) {
        out[0] = (first == INT32_MAX) ? 0 : err[first];
        out[1] = (first == INT32_MAX) ? -1 : first;
    }
}

void launch_first_error(const int32_t* err, int32_t batch, int32_t* out, hipStream_t s)
{
    hipLaunchKernelGGL(first_error_kernel, dim3(1), dim3(1024), 0, s, err, batch, out);
}

void launch_ctrl_reset(const CtrlArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(ctrl_reset_kernel, dim3(64), dim3(256), 0, s, a);
}

void launch_ctrl_begin(const CtrlArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(ctrl_begin_kernel, dim3(1), dim3(1024), 0, s, a);
}

void launch_copy_back(const CopyArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(copy_back_kernel, dim3(1024, a.ngroups), dim3(256), 0, s, a);
}

}  // namespace fvk
