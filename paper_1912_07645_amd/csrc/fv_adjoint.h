// fv_adjoint.h -- discrete adjoint kernels (internal).
#pragma once

#include "fv_common.h"

namespace fvk {

// One reverse Runge--Kutta stage. With the forward stage
//   U^(s) = (1 - beta) U^n + beta (U^(s-1) + dt L(U^(s-1))),
// and lam = dQ/dU^(s), it computes
//   prev = beta (lam + dt J(U^(s-1))^T lam)      (the adjoint of U^(s-1)),
//   acc  = acc + (1 - beta) lam                    (the adjoint of U^n, accumulated),
// where J = dL/dU uses the forward pass's branch choices. mode 0: acc is initialised
// (first reverse stage of a step); mode 1: accumulated; mode 2 (the stage whose input is
// U^n itself): prev = acc + beta (lam + dt J^T lam) is the adjoint of U^n.
struct AdjArgs {
    const double* U;       // U^(s-1) [batch][NF][cells]
    const double* lam;     // dQ/dU^(s)
    double* prev;          // out
    double* acc;           // in/out (modes 0, 1); read in mode 2
    int64_t cells;
    int32_t n[3];
    int32_t tiles[3];
    int32_t ntiles;
    int32_t batch;
    int32_t bc[3];
    int32_t mode;
    double beta;
    double dt;
    int64_t nblocks;
    Phys ph;
    // branch signature (diagnostic; null: off): sig[sample] += one hashed term per face of the
    // launch, from salt (the launch), the face and its branch choices, modulo 2^64
    unsigned long long* sig;
    unsigned long long salt;
};

struct AdjKernel {
    void (*launch)(const AdjArgs&, hipStream_t);
    int32_t bx, by, bz;
};

// Adjoint stage kernel for (dim, reconstruction) with the Euler equations and the Rusanov
// flux; nullptr if not available.
const AdjKernel* find_adjoint_kernel(int dim, int eq, int recon, int flux);

// Kinetic energy integrated over the cells whose index along axis 1 lies in [j0, j1):
// Q[b] = (dx dy ...) sum 0.5 ((m . m) (1 / rho)), and (if grad != nullptr)
// grad[b] = seed[b] dQ/dU (zero outside the band).
void launch_qoi_ke(const double* state, int32_t dim, const int32_t n[3], int32_t batch,
                   int32_t j0, int32_t j1, double volume, const double* seed, double* Q,
                   double* grad, double* partial, int32_t nblk, hipStream_t s);
int qoi_blocks(int64_t cells);

// out[b][k] = sum_lines (sum_{cells of the line} sum_q lam[b][q][cell] D[b][q][cell])
//             * E[b][line][k], lines = the rows along axis 1 (fixed x and z), summed in
// fixed order. line_sums: scratch [batch][lines].
void launch_line_vjp(const double* lam, const double* D, const double* E, int32_t nf,
                     const int32_t n[3], int32_t batch, int32_t ntheta, double* line_sums,
                     double* out, hipStream_t s);

}  // namespace fvk
