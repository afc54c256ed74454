// fv_small.h -- the single-workgroup time loop for small 1D grids (fv_small.hip).
#pragma once

#include "fv_common.h"

namespace fvk {

struct SmallArgs {
    double* state;             // [batch][NF][n], updated in place
    int64_t batch;
    int32_t n;                 // cells
    int32_t bc;                // boundary condition of the axis
    Phys ph;
    double* t;                 // [batch] in/out (unused when fixed)
    int64_t* steps;            // [batch] step counts, kept across launches
    int32_t* err;              // [batch] status
    int32_t* running;          // [batch] still evolving, kept across launches
    int32_t* n_running;        // samples still running after this launch (added to)
    int64_t chunk;             // at most this many steps per sample in one launch
    int32_t first;             // first launch of a run: steps, err and running start afresh
    double t_end, cfl;
    int64_t max_steps;
    int32_t limit_is_error;    // reaching max_steps before t_end is an error
    int32_t fixed;             // fixed step size fixed_dt, checked against cfl_bound
    double fixed_dt, cfl_bound;
    int32_t nst;               // Runge--Kutta stages
    double beta[3];            // stage weights
};

struct SmallKernel {
    int32_t eq, recon, flux;
    void (*launch)(const SmallArgs&, hipStream_t);
    int32_t max_cells;         // largest grid the workgroup's LDS and registers hold
};

// The single-workgroup kernel for a 1D scheme, or null if none is built for it.
const SmallKernel* find_small_kernel(int eq, int recon, int flux);

}  // namespace fvk
