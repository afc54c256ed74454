/*
 * fv.h -- C ABI of libfv, an MI355X (gfx950) library for the explicit finite-volume
 * method of Lye, "Alsvinn: A fast multi-GPGPU finite volume solver with a strong emphasis on
 * reproducibility" (arXiv:1912.07645), and its on-device Monte Carlo statistics.
 *
 * The method (Section 2.1): solve u_t + div F(u) = 0 on D x [0, T], u(x, 0) = u_0 (eq. 1.1)
 * through the semi-discrete scheme d/dt U_i + sum_k (F_{i+1/2 e_k} - F_{i-1/2 e_k}) / dx_k
 * = 0 (eq. 2.1), with a numerical flux (Rusanov, HLL, HLLC), a reconstruction of the face
 * values (piecewise constant, MUSCL with the minmod limiter, third-order WENO) and a strong
 * stability preserving Runge--Kutta stepper. Section 2.2: Monte Carlo estimates
 * (1/M) sum_k G(u_k) over samples, with per-cell mean and variance and two-point structure
 * functions computed on the GPU.
 *
 * Conventions shared by every entry point:
 *   - All floating-point data is IEEE binary64.
 *   - State arrays are device memory in structure-of-arrays layout
 *     [batch][field][nz][ny][nx], x fastest, densely packed (unused axes have extent 1).
 *     Euler fields are (rho, m_x[, m_y[, m_z]], E); scalar equations have one field.
 *   - Device arrays passed in are owned by the caller and must stay valid until the call
 *     returns. The library owns only its opaque handles and any workspace it allocates
 *     itself; it never frees caller memory.
 *   - Work is ordered on the solver's stream (fv_set_stream). Calls that poll device flags
 *     (fv_evolve, fv_advance, fv_evolve_fixed_dt) return after the device has finished.
 *   - Every function returns fv_status (or a plain value where stated). On failure a
 *     description is available from fv_last_error() in the calling thread. Argument errors
 *     are found on the host before any device work is enqueued. No C++ exception crosses the
 *     boundary.
 *   - Results are bit-for-bit reproducible from run to run and independent of the batch
 *     size, the number of samples per launch and the tile shape chosen by the tuner.
 */
#ifndef FV_H
#define FV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FV_OK = 0,
    FV_EINVAL = 1,      /* bad argument: null pointer, size <= 0, cfl outside (0, 1], ...   */
    FV_ENOTSUP = 2,     /* valid but unsupported combination (HLLC for a scalar equation)   */
    FV_ENOMEM = 3,      /* device or host allocation failed, or workspace too small         */
    FV_EDEVICE = 4,     /* a HIP runtime call failed                                        */
    FV_ENONPHYS = 5,    /* a sample reached rho <= 0, p <= 0 or a non-finite value          */
    FV_EMAXSTEPS = 6,   /* a sample did not reach t_end within max_steps steps              */
    FV_ECFL = 7         /* fixed-dt run: dt * max wave speed / dx exceeded the bound        */
} fv_status;

typedef enum { FV_BC_PERIODIC = 0, FV_BC_TRANSMISSIVE = 1 } fv_bc;
typedef enum { FV_EQ_ADVECTION = 0, FV_EQ_BURGERS = 1, FV_EQ_EULER = 2,
               FV_EQ_SHALLOW_WATER = 3, FV_EQ_MHD = 4 } fv_eq_kind;
/* Numerical fluxes (Section 2.1 names HLLC, Godunov, Rusanov, Roe and entropy-conservative
 * fluxes): Rusanov (local Lax--Friedrichs); HLL and HLLC with Davis wave speeds; Roe with
 * Roe's average state and Harten's entropy fix on the acoustic waves (for Burgers the Roe
 * speed (uL + uR)/2 with the fix over a rarefaction fan, for advection upwinding); EC, the
 * two-point entropy-conservative flux: Tadmor's (uL^2 + uL uR + uR^2)/6 for Burgers,
 * Chandrashekar's (logarithmic means of rho and rho/(2p)) for Euler; EC4, the fourth-order
 * entropy-conservative flux of LeFloch, Mercier and Rohde, (4/3) EC(U_i, U_i+1) -
 * (1/6) (EC(U_i, U_i+2) + EC(U_i-1, U_i+1)) on the cell values, which requires
 * FV_RECON_FIRST_ORDER (no reconstruction; FV_ENOTSUP otherwise); both EC fluxes are for
 * Burgers and Euler only, and the Euler ones call log1p(), so they agree with other
 * implementations to rounding; GODUNOV, the
 * physical flux of the exact Riemann solution at the face (Euler: Toro's star pressure by
 * Newton's method and wave sampling; Burgers: the entropy solution; advection: upwinding),
 * not for shallow water. The Euler Godunov flux calls pow() and stops Newton's method on a
 * step-size test, so it agrees with other implementations to rounding, not bit for bit. */
typedef enum { FV_FLUX_RUSANOV = 0, FV_FLUX_HLL = 1, FV_FLUX_HLLC = 2, FV_FLUX_ROE = 3,
               FV_FLUX_EC = 4, FV_FLUX_GODUNOV = 5, FV_FLUX_EC4 = 6 } fv_flux;
/* Reconstructions (Section 2.1 names ENO and WENO): piecewise constant; MUSCL with the
 * minmod limiter; third-order WENO; second-order ENO (the one-sided difference of smaller
 * magnitude, the left one on a tie). Component-wise on the conserved variables. */
typedef enum { FV_RECON_FIRST_ORDER = 0, FV_RECON_MUSCL_MINMOD = 1, FV_RECON_WENO3 = 2,
               FV_RECON_ENO2 = 3 } fv_recon;
typedef enum { FV_INT_FORWARD_EULER = 0, FV_INT_SSPRK2 = 1, FV_INT_SSPRK3 = 2 } fv_integrator;

/* Uniform Cartesian grid on [lo, hi] per axis (Section 2.1: cells i with averages U_i).
 * dim in 1..3; n[k] >= 1 cells on axis k, and n[k] == 1 for k >= dim; bc[k] is the
 * boundary condition on both ends of axis k (periodic wrap, or transmissive: every ghost
 * layer copies the edge cell). */
typedef struct {
    int32_t dim;
    int32_t bc[3];
    int64_t n[3];
    double lo[3];
    double hi[3];
} fv_grid;

/* The flux function F of eq. (1.1): linear advection F = a u (velocity[k] = a_k), Burgers
 * F = u^2/2 in every direction, the compressible Euler equations with the gamma law
 * p = (gamma - 1)(E - |m|^2 / (2 rho)) (gamma > 1), or the shallow-water equations
 * (h, hu_1..hu_dim) with flux along k (hu_k, hu u_k + g h^2 / 2 e_k), u = hu (1/h),
 * gravity = g > 0, in 1D and 2D (a second workload family; the paper's framework is built
 * for several equations, Section 2.1), or ideal MHD (the introduction names it among the
 * systems of eq. 1.1): eight fields (rho, m_x, m_y, m_z, E, B_x, B_y, B_z) in every dimension,
 * p = (gamma - 1)(E - |m|^2 / (2 rho) - |B|^2 / 2), flux along k (m_k, m u_k - B_k B +
 * (p + |B|^2/2) e_k, (E + p + |B|^2/2) u_k - B_k (u . B), u_k B - B_k u), with the Rusanov
 * and HLL fluxes on the fast magnetosonic speed only (FV_ENOTSUP otherwise) and no
 * divergence cleaning. Statistics of MHD take (rho, u_x, u_y, u_z, E, B_x, B_y, B_z). */
typedef struct {
    int32_t kind;          /* fv_eq_kind */
    double gamma;
    double velocity[3];
    double gravity;        /* shallow water only */
} fv_equation;

typedef struct fv_solver fv_solver;   /* opaque, library-owned */
typedef struct fv_stats fv_stats;     /* opaque, library-owned */
typedef struct fv_adjoint fv_adjoint; /* opaque, library-owned */

/* ------------------------------------------------------------------ solver lifetime */

/* Create a solver for one grid, equation and scheme (Section 2.1: numerical flux, face
 * reconstruction, SSP Runge--Kutta stepper). flux, recon, integrator take the enum values
 * above. *out receives the handle. FV_ENOTSUP for HLLC with a scalar equation; FV_EINVAL
 * for any malformed grid or enum, or a grid of more than 2^31 - 1 cells; FV_EDEVICE if no
 * gfx950 device is current. */
fv_status fv_create(const fv_grid* grid, const fv_equation* eq, int32_t flux, int32_t recon,
                    int32_t integrator, fv_solver** out);

/* Destroy a solver and the workspace it allocated itself. NULL is accepted. */
fv_status fv_destroy(fv_solver* solver);

/* Order the solver's device work after, and before, work on this HIP stream (hipStream_t
 * passed as void*; NULL means the null stream). Default: the null stream. */
fv_status fv_set_stream(fv_solver* solver, void* hip_stream);

/* Number of conserved fields: dim + 2 for Euler, 1 for scalar equations; -1 on NULL. */
int32_t fv_num_fields(const fv_solver* solver);

/* Bytes of device workspace that fv_evolve / fv_advance / fv_evolve_fixed_dt need for a
 * batch of `batch` samples (Runge--Kutta stage copies and per-sample control words). */
fv_status fv_workspace_size(const fv_solver* solver, int64_t batch, size_t* bytes);

/* Hand the solver caller-owned device memory (256-byte aligned) to use as workspace
 * instead of allocating its own. dev_ptr = NULL returns to library-allocated workspace.
 * A later call whose batch needs more than `bytes` fails with FV_ENOMEM. */
fv_status fv_set_workspace(fv_solver* solver, void* dev_ptr, size_t bytes);

/* ------------------------------------------------------------------ time stepping */

/* Evolve each sample b of state (device double[batch][fields][cells], updated in place)
 * from t[b] to t_end (device double[batch], in/out) with explicit SSP Runge--Kutta steps of
 * eq. (2.1). Each step of sample b uses dt_b = cfl / M_b, with M_b = max over cells and axes
 * of (|u_k| + c) / dx_k (Euler), |u| / dx_k (Burgers), |a_k| / dx_k (advection), evaluated
 * on the state the step starts from; the last step is clipped to end exactly at t_end.
 * Samples advance independently (per-sample dt). Before every step, and at the end, the
 * state is checked: rho <= 0, p <= 0 or a non-finite value stops that sample with
 * FV_ENONPHYS. A sample that needs more than max_steps steps stops with FV_EMAXSTEPS.
 * steps (device int64[batch], may be NULL) receives the number of steps taken; err
 * (device int32[batch], may be NULL) the per-sample status. Returns FV_OK if every sample
 * reached t_end, otherwise the first failing sample's status. cfl must lie in (0, 1]. */
fv_status fv_evolve(fv_solver* solver, double* state, int64_t batch, double* t, double t_end,
                    double cfl, int64_t max_steps, int64_t* steps, int32_t* err);

/* As fv_evolve, but take at most nsteps steps per sample and treat stopping early as
 * success: a sample that has not reached t_end after nsteps steps keeps err = FV_OK. */
fv_status fv_advance(fv_solver* solver, double* state, int64_t batch, double* t, double t_end,
                     double cfl, int64_t nsteps, int64_t* steps, int32_t* err);

/* For callers that cannot allocate device memory (code under stream capture, tight serving
 * loops, harnesses that forbid hipMalloc): fv_advance with the same arguments, semantics and
 * results (bit for bit), run in a workspace that the library holds in a fixed device array,
 * one per device, for the life of the process, instead of the solver's workspace. The call
 * allocates no device or pinned host memory: it launches the tiled stage kernels directly
 * (no graph, no single-workgroup variant, no kernel timing) and finds the first failing
 * sample on the device. The batch's workspace (fv_workspace_size) must fit in
 * fv_noalloc_capacity() bytes (68 MiB: e.g. one 1024^2 Euler sample with SSP-RK3, or 16
 * samples of 256^2), else FV_ENOMEM before any device work. Every solver on a device shares
 * that device's array, which keeps the last call's contents (each call initialises what it
 * reads): calls that overlap in time on one device race and give undefined results. */
fv_status fv_advance_noalloc(fv_solver* solver, double* state, int64_t batch, double* t,
                             double t_end, double cfl, int64_t nsteps, int64_t* steps,
                             int32_t* err);

/* Bytes of the fixed per-device workspace of fv_advance_noalloc. */
size_t fv_noalloc_capacity(void);

/* Exactly nsteps steps of the fixed size dt for every sample (no clipping). Before each
 * step a sample whose dt * M_b exceeds cfl_bound stops with FV_ECFL; non-physical states
 * stop it with FV_ENONPHYS. err as in fv_evolve. */
fv_status fv_evolve_fixed_dt(fv_solver* solver, double* state, int64_t batch, double dt,
                             int64_t nsteps, double cfl_bound, int32_t* err);

/* Several solvers (grids of different resolution sharing one equation and scheme, e.g. the
 * levels of a multilevel Monte Carlo estimate, Section 2.2) evolved together: every
 * Runge--Kutta stage of all groups runs as one launch, each sample with its own time step.
 * Group g (1 <= n_groups <= 8) has solvers[g] (distinct solvers), its batch
 * states[g][batches[g]][fields][cells], times t[g] (device double[batches[g]]), step counts
 * steps[g] (device int64[batches[g]]) and statuses err[g] (device int32[batches[g]]); steps
 * and err, and their entries, may be NULL. All solvers must share dimension, boundary
 * conditions, equation, flux, reconstruction, integrator and tile; the work runs on
 * solvers[0]'s stream. Semantics per sample as in fv_evolve. */
fv_status fv_evolve_multi(int32_t n_groups, fv_solver* const* solvers, double* const* states,
                          const int64_t* batches, double* const* t, double t_end, double cfl,
                          int64_t max_steps, int64_t* const* steps, int32_t* const* err);

/* ------------------------------------------------------------------ tile tuning */

/* Tile shapes: each (dimension, equation, reconstruction, flux) has one or more compiled
 * tile shapes ("variants"), all producing bit-identical results. A 1D grid small enough for
 * one workgroup's LDS (with two ghost layers: Euler up to 1277 cells, shallow water 1917,
 * ideal MHD 477, scalar equations 3837; every flux but the fourth-order EC one) has one
 * more, last variant: the whole time loop of each
 * sample in one workgroup (state in LDS, the step decision on the chip, one launch per
 * 65 536 steps), for latency-bound small problems; its tile is the whole grid. Step
 * profiling (fv_profile_enable) and fv_evolve_multi use the tiled kernels.
 * fv_num_variants returns their number (-1 on NULL); fv_set_variant selects one (FV_EINVAL
 * if out of range); fv_get_tile reports the current tile shape in cells and its variant
 * index (any output may be NULL). */
int32_t fv_num_variants(const fv_solver* solver);
fv_status fv_set_variant(fv_solver* solver, int32_t variant);
fv_status fv_get_tile(const fv_solver* solver, int32_t* bx, int32_t* by, int32_t* bz,
                      int32_t* variant);

/* Autotuner: after about 50 ms of untimed warm-up steps, time runs of 4 to 32 whole steps
 * (about 8 ms each) of every variant on a copy of `state` (device, [batch][fields][cells],
 * not modified) and select the one with the fastest median run; *chosen (may be NULL)
 * receives it. reps < 1 means 3 timed runs per variant. Allocates a copy of the state for the
 * duration of the call; on an error the variant selected before the call is kept. */
fv_status fv_tune(fv_solver* solver, double* state, int64_t batch, int32_t reps,
                  int32_t* chosen);

/* ------------------------------------------------------------------ kernel timing */

/* Kernel timing for roofline measurements. While enabled (on != 0), the time-stepping
 * calls enqueue their launches directly instead of replaying a graph, and bracket each
 * step's Runge--Kutta stage launches, which follow each other directly, with one pair of HIP
 * events on the solver's internal stream; enabling or disabling resets the totals.
 * fv_profile_read returns the accumulated device time of the stage launches in milliseconds
 * and their number (outputs may be NULL). Launches of samples that had already finished count
 * as well (they return immediately). */
fv_status fv_profile_enable(fv_solver* solver, int32_t on);
fv_status fv_profile_read(const fv_solver* solver, double* stage_ms, int64_t* stage_launches);

/* ------------------------------------------------------------------ statistics */

/* Running Monte Carlo statistics (Section 2.2) on the solver's grid. Quantities: Euler
 * (rho, u_1..u_dim, E) with u_k = m_k * (1/rho); shallow water (h, u_1..u_dim) with
 * u_k = hu_k * (1/h); ideal MHD (rho, u_x, u_y, u_z, E, B_x, B_y, B_z) with
 * u_k = m_k * (1/rho); scalar equations the field itself.
 * max_h >= 0 is the largest lag of the second-order structure function
 * S_q(h) = 1/(dim N) sum_axes sum_x (q(x + h e_axis) - q(x))^2 (periodic grids only,
 * max_h < n[k] on every axis; FV_ENOTSUP otherwise). */
fv_status fv_stats_create(const fv_solver* solver, int32_t max_h, fv_stats** out);

/* Add the samples of state (device double[batch][fields][cells]) in index order:
 * per-cell Welford updates of the mean and M2 of every quantity, and Welford updates over
 * samples of S_q(h), h = 1..max_h. Stream-ordered on the solver's stream. */
fv_status fv_stats_accumulate(fv_stats* stats, const double* state, int64_t batch);

/* Copy the statistics into caller device memory (any pointer may be NULL):
 * mean, var: double[quantities][cells] (var = M2 / count, population variance);
 * s2_mean, s2_var: double[quantities][max_h]; count: host int64. Synchronises. */
fv_status fv_stats_read(const fv_stats* stats, double* mean, double* var, double* s2_mean,
                        double* s2_var, int64_t* count);

/* Multilevel Monte Carlo (Section 2.2): sum_l (1/M_l) sum_k (G(u^l_k) - G(u^{l-1}_k)).
 * fv_stats_accumulate_diff adds coupled samples (the same random input evolved on the
 * stats' fine grid and on a coarser grid) in index order: per fine cell, Welford updates of
 * x = q(u_fine) - P q(u_coarse), where P copies each coarse cell onto the fine cells it
 * contains (piecewise-constant prolongation). fine: device double[batch][fields][fine
 * cells]; coarse_state: device double[batch][fields][coarse cells] on coarse's grid, which
 * must divide the fine grid on every axis (FV_EINVAL otherwise); the stats must have max_h
 * = 0 (FV_ENOTSUP otherwise). The first level (u^0 = 0) uses fv_stats_accumulate. */
fv_status fv_stats_accumulate_diff(fv_stats* stats, const double* fine, const fv_solver* coarse,
                                   const double* coarse_state, int64_t batch);

/* The multilevel estimate on the finest grid: out[q][cell] = sum_{l = 1..L} P_{l -> L}
 * mean_l, with levels[0..L-1] ordered coarse to fine (levels[L-1] on the finest grid) and
 * added in that order. out: device double[quantities][finest cells]. Synchronises. */
fv_status fv_mlmc_combine(int32_t nlevels, const fv_stats* const* levels, double* out);

/* Reset to zero samples. */
fv_status fv_stats_reset(fv_stats* stats);

fv_status fv_stats_destroy(fv_stats* stats);

/* ------------------------------------------------------------------ PDFs and shell structure functions */

/* Point PDFs (Section 2.2 lists them among the statistics, after Fjordholm, Lye and Mishra):
 * for every cell points[i] (host int64 array of npoints cell indices, x fastest), the
 * histogram over the batch's samples of one quantity (as for fv_stats_create: Euler rho,
 * u_1..u_dim, E with u_k = m_k * (1/rho); shallow water h, u_1..u_dim; ideal MHD rho,
 * u_x, u_y, u_z, E, B_x, B_y, B_z; scalar equations the field, quantity 0) at that
 * cell. nbins equal bins on [lo, hi): a value v in range goes to bin
 * floor(((v - lo) / (hi - lo)) * nbins) computed in FP64 in that order, or to the last bin
 * if that rounds to nbins. counts: device int64 [npoints][nbins + 2], ADDED to (the caller
 * clears it): the bins, then one counter for values below lo and one for values not below hi
 * (NaN included). Exact integer counts, independent of launch order. state: device
 * double[batch][fields][cells]. FV_EINVAL: a NULL pointer, batch < 1, npoints < 0, no such
 * quantity, nbins outside 1..65536, !(lo < hi), a cell index outside the grid. Stream-ordered;
 * `points` may be reused when the call returns. */
fv_status fv_point_pdf(const fv_solver* solver, const double* state, int64_t batch,
                       int32_t quantity, int64_t npoints, const int64_t* points, double lo,
                       double hi, int32_t nbins, int64_t* counts);

/* Joint PDFs: for every pair (pairs[i][0], pairs[i][1]) of cells (host int64 [npairs][2]),
 * the histogram over samples of (quantity_a at the first cell, quantity_b at the second) on
 * nbins x nbins bins of [lo_a, hi_a) x [lo_b, hi_b), each axis binned as in fv_point_pdf.
 * counts: device int64 [npairs][nbins * nbins + 1], ADDED to: bin ka * nbins + kb, then one
 * counter for pairs with either value outside its range. Errors as for fv_point_pdf. */
fv_status fv_joint_pdf(const fv_solver* solver, const double* state, int64_t batch,
                       int32_t quantity_a, int32_t quantity_b, int64_t npairs,
                       const int64_t* pairs, double lo_a, double hi_a, double lo_b,
                       double hi_b, int32_t nbins, int64_t* counts);

/* Structure functions over cube or ball shells (the two-point structure functions of
 * Section 2.2 in the averaged form of Fjordholm, Lye and Mishra), per sample:
 * out[b][q][h - 1] = S_p(h) = 1/(N |A_h|) sum_{o in A_h} sum_x |q(x + o) - q(x)|^p for
 * h = 1..max_h on the periodic grid, p = order in {1, 2}, with the cube shell
 * A_h = {o : max_k |o_k| = h} (ball = 0) or the ball shell {o : (h-1)^2 < |o|^2 <= h^2}
 * (ball = 1), o over the grid's axes. out: device double [batch][quantities][max_h].
 * Sums are taken per cell over the shell, then over cells; they agree with the definition's
 * order to rounding. FV_EINVAL: a NULL pointer, batch < 1, max_h outside 1..64, order or ball
 * out of range. FV_ENOTSUP: a non-periodic axis, max_h >= cells of an axis, or a tile with its
 * halo beyond 64 KB of LDS (3D: max_h <= 6; 2D: max_h <= 36). Stream-ordered. */
fv_status fv_structure_shell(const fv_solver* solver, const double* state, int64_t batch,
                             int32_t max_h, int32_t order, int32_t ball, double* out);

/* ------------------------------------------------------------------ discrete adjoint */

/* Discrete adjoint of a fixed-step run (not in the paper; it differentiates the scheme of
 * Section 2.1). The forward map is nsteps SSP Runge--Kutta steps of size dt; the adjoint is
 * the exact transpose of its linearisation, with the forward pass's branch choices (the
 * larger Rusanov wave speed, ties to the right state; the minmod argument selected; the
 * derivative of |u| at 0 taken as 0). Supported: the Euler equations in 1D and 2D on periodic
 * grids with the Rusanov flux and first-order or MUSCL-minmod reconstruction (FV_ENOTSUP
 * otherwise, also for a transmissive axis).
 *
 * fv_adjoint_create allocates, for `batch` samples of the solver's grid, ceil(nsteps/every)
 * checkpoint states, every * stages + 1 segment states and three adjoint states (device
 * memory owned by the handle). every <= 0 selects ceil(sqrt(nsteps)). cfl_bound is checked
 * over the whole forward trajectory (dt * max wave speed). */
fv_status fv_adjoint_create(fv_solver* solver, int64_t batch, int64_t nsteps, double dt,
                            int64_t every, double cfl_bound, fv_adjoint** out);

/* The same adjoint with binomial checkpointing (Griewank's revolve schedule) instead of
 * segments: the forward run keeps only the initial state, and the reverse sweep places up to
 * `snapshots` (>= 0) further checkpoints where the binomial schedule puts them. Reversing
 * nsteps = l steps then runs p + l forward steps (l = one stage recomputation per step when
 * the stepper has more than one stage, 0 otherwise), p = t l - C(snapshots + 1 + t, t - 1)
 * with t the smallest integer such that C(snapshots + 1 + t, t) >= l (p = l (l - 1) / 2 for
 * snapshots = 0): the fewest for that memory. Device memory: snapshots + stages + 5 states
 * per batch instead of the segments' ceil(nsteps / every) + every * stages + 4. Same
 * arguments, errors and gradient (bit for bit) as fv_adjoint_create otherwise. */
fv_status fv_adjoint_create_binomial(fv_solver* solver, int64_t batch, int64_t nsteps, double dt,
                                     int64_t snapshots, double cfl_bound, fv_adjoint** out);

/* Forward steps the last fv_adjoint_backward of this handle ran to recompute states (host
 * int64 out). */
fv_status fv_adjoint_recomputed_steps(const fv_adjoint* adj, int64_t* steps);

/* Forward run from state0 (device, [batch][fields][cells], not modified) to stateT (device,
 * same shape), storing checkpoints. FV_ENONPHYS / FV_ECFL if a sample's trajectory left the
 * physical states or the CFL bound. */
fv_status fv_adjoint_forward(fv_adjoint* adj, const double* state0, double* stateT);

/* Reverse sweep: dQ/dU0 (device, [batch][fields][cells], written) from dQ/dUT (device, same
 * shape, not modified), recomputing each checkpoint segment. Needs a completed
 * fv_adjoint_forward. */
fv_status fv_adjoint_backward(fv_adjoint* adj, const double* dQ_dUT, double* dQ_dU0);

/* Branch signature (a diagnostic for finite-difference checks of the adjoint, whose map is only
 * piecewise smooth): while sig (device uint64[batch], caller-owned and cleared by the caller)
 * is set, every fv_adjoint_backward adds to sig[b], modulo 2^64, one hashed term per face and
 * reverse Runge--Kutta stage of sample b. The term hashes the stage's place in the sweep, the
 * face, and the branches the forward pass took there: the minmod branch of both face values
 * of every field, the side of the larger Rusanov speed, the sign of the selected normal
 * velocity. Two trajectories that take the same branches everywhere give equal signatures;
 * one differing branch changes the signature except with probability about 2^-64. Both
 * checkpointing schedules give the same signature. sig = NULL turns it off. */
fv_status fv_adjoint_set_signature(fv_adjoint* adj, uint64_t* sig);

fv_status fv_adjoint_destroy(fv_adjoint* adj);

/* Quantity of interest: the kinetic energy sum 0.5 |m|^2 / rho times the cell volume, over the
 * cells whose index along axis 1 lies in [j0, j1) (all cells of those rows), per sample:
 * Q[b] (device double[batch], may be NULL). If dQ_dU (device, state-shaped) is given, it
 * receives seed[b] * dQ[b]/dU (seed: device double[batch], required then), zero outside the
 * band. Euler equations only. Sums use a fixed order (reproducible). */
fv_status fv_qoi_kinetic_energy(fv_solver* solver, const double* state, int64_t batch, int64_t j0,
                                int64_t j1, const double* seed, double* Q, double* dQ_dU);

/* Chain rule through initial data that depends on parameters theta through one scalar per
 * line along axis 1 (a line: fixed x and z indices, e.g. the displaced interface of a shear
 * layer): out[b][k] = sum_lines (sum_{cells of the line} sum_fields lambda0 * dU_dline)
 * * dline_dtheta[b][line][k]. lambda0, dU_dline: device [batch][fields][cells];
 * dline_dtheta: device [batch][lines = n[2] * n[0], z slowest][ntheta]; out: device
 * [batch][ntheta]. Fixed summation order. */
fv_status fv_line_vjp(fv_solver* solver, const double* lambda0, const double* dU_dline,
                      const double* dline_dtheta, int32_t ntheta, int64_t batch, double* out);

/* ------------------------------------------------------------------ split-buffer decomposition */

/* Domain decomposition of one solver's grid into parts[0] x parts[1] x parts[2] equal
 * subdomains with their own state arrays on this device, advanced with a halo exchange every
 * Runge--Kutta stage: the communication of a multi-GPU run (Section 2.1: the exchange and the
 * compactification of the boundary data are overlapped with the computation of the inner
 * domain; Section 3.1: splits along x, along y, along both), emulated with device-to-device
 * copies. Each subdomain stores G ghost layers (2 for MUSCL and WENO3) on every split axis.
 * Each stage packs the G owned layers next to every face of every subdomain into one
 * contiguous message per (subdomain, split axis, side). It copies each message on a second
 * stream into a receive buffer and unpacks it into the neighbour's ghost layers. Results are
 * bit for bit those of the unsplit solver (the per-cell arithmetic is the same, and the
 * maximum wave speed is merged exactly over the subdomains).
 *
 * fv_decomp_create: parts[k] >= 1 must divide n[k], parts[k] = 1 beyond the grid's dimension,
 * at most 8 subdomains, split axes periodic with at least 2 G cells per subdomain; the SSP-RK2 or
 * SSP-RK3 stepper; the Euler equations with WENO3 + HLLC (2D, 3D) or MUSCL + HLL or MUSCL +
 * Rusanov (2D) (FV_ENOTSUP otherwise, FV_EINVAL for bad sizes). It allocates the subdomain
 * arrays (cleared) for `batch` samples and the message buffers. The handle uses the solver's
 * stream and must not outlive the solver; batch 1..8192. */
typedef struct fv_decomp fv_decomp;  /* opaque, library-owned */
fv_status fv_decomp_create(fv_solver* solver, const int32_t* parts, int64_t batch,
                           fv_decomp** out);

/* Copy a whole-grid state (device double[batch][fields][cells]) into the subdomains' owned
 * cells (scatter), or the owned cells back into a whole-grid state (gather). Stream-ordered. */
fv_status fv_decomp_scatter(fv_decomp* d, const double* state);
fv_status fv_decomp_gather(fv_decomp* d, double* state);

/* fv_advance on the subdomains: at most nsteps steps per sample, each with dt = cfl / M_b and
 * the last clipped at t_end (t: device double[batch], in/out; steps: device int64[batch] out,
 * err: device int32[batch] out, both may be NULL). mode is FV_DECOMP_OVERLAP and/or
 * FV_DECOMP_DMA, or 0. With 0, every stage exchanges the halos, then updates every tile.
 * FV_DECOMP_OVERLAP: every stage packs and starts the copies, then updates the interior tiles
 * (whose reads stay in owned cells) on the solver's stream, while the copy stream carries out
 * the copies, the unpacking and the update of the boundary shell; the next stage waits for
 * both. FV_DECOMP_DMA: the copies run on the DMA engines (hipMemcpyDeviceToDeviceNoCU), as
 * transfers between GPUs would, instead of copy kernels on the compute units. FV_EINVAL for
 * any other mode. Returns FV_OK or the first failing sample's status, after the device has
 * finished. */
enum { FV_DECOMP_OVERLAP = 1, FV_DECOMP_DMA = 2 };
fv_status fv_decomp_advance(fv_decomp* d, double* t, double t_end, double cfl, int64_t nsteps,
                            int64_t* steps, int32_t* err, int32_t mode);

/* Timing: while enabled, fv_decomp_advance records events around every whole step (compute
 * stream) and around every stage's copies (copy stream). fv_decomp_profile_read returns their
 * accumulated durations in milliseconds and the number of timed steps (outputs may be NULL);
 * enabling or disabling resets them. */
fv_status fv_decomp_profile_enable(fv_decomp* d, int32_t on);
fv_status fv_decomp_profile_read(const fv_decomp* d, double* step_ms, double* copy_ms,
                                 int64_t* steps);

/* Layout facts (outputs may be NULL): subdomains, messages per stage, bytes of all messages of
 * one stage, tiles per subdomain in the interior box and in the boundary shell. */
fv_status fv_decomp_info(const fv_decomp* d, int32_t* nsub, int32_t* messages,
                         int64_t* halo_bytes, int32_t* interior_tiles, int32_t* shell_tiles);

fv_status fv_decomp_destroy(fv_decomp* d);

/* ------------------------------------------------------------------ misc */

/* Human-readable description of the last failure in this thread ("" if none). Valid until
 * the next fv_* call in the same thread. */
const char* fv_last_error(void);

/* Arithmetic self-check: quot[i] = a[i] / b[i], root[i] = sqrt(a[i]) on the device with the
 * same division and square root the kernels use (all device arrays of n doubles), so that
 * tests can compare them bit for bit with correctly rounded host results. Synchronises. */
fv_status fv_check_arith(const double* a, const double* b, double* quot, double* root,
                         int64_t n);

/* Library version string. */
const char* fv_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FV_H */
