// fv_control.h -- device-side step control (internal).
#pragma once

#include "fv_common.h"

namespace fvk {

struct CtrlGroup {
    double* t;                  // [batch] current time (adaptive mode)
    double* dt;                 // [batch]
    int32_t* running;           // [batch]
    int32_t* active;            // [batch]
    unsigned long long* mbits;  // [kSpeedSlots][speed_pitch(batch)]
    int32_t* bad;               // [batch]
    int64_t* steps;             // [batch]
    int32_t* err;               // [batch]
    int32_t batch;
};

struct CtrlArgs {
    CtrlGroup g[kMaxGroups];
    int32_t ngroups;
    int32_t fixed;           // fixed-dt mode
    int32_t limit_is_error;  // max_steps reached before t_end is FV_EMAXSTEPS
    double t_end;
    double cfl;
    double fixed_dt;
    double cfl_bound;
    int64_t max_steps;
    int32_t* n_running;      // out: [0] samples taking the step just decided, [1 + g] per group
};

struct CopyGroup {
    const double* src;
    double* dst;
    const int32_t* active;
    int64_t per_sample;      // doubles per sample
    int32_t batch;
};

struct CopyArgs {
    CopyGroup g[kMaxGroups];
    int32_t ngroups;
};

void launch_ctrl_reset(const CtrlArgs& a, hipStream_t s);
void launch_ctrl_begin(const CtrlArgs& a, hipStream_t s);
void launch_copy_back(const CopyArgs& a, hipStream_t s);
// out: device int32[2] = (status of the first failing sample, its index), or (0, -1).
void launch_first_error(const int32_t* err, int32_t batch, int32_t* out, hipStream_t s);

}  // namespace fvk
