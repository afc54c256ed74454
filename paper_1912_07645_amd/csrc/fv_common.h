// fv_common.h -- internal types shared by the host side of libfv and its kernel
// instantiation units. Not part of the public ABI (that is include/fv.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fvk {

enum { EQ_ADVECTION = 0, EQ_BURGERS = 1, EQ_EULER = 2, EQ_SWE = 3, EQ_MHD = 4 };
enum { FLUX_RUSANOV = 0, FLUX_HLL = 1, FLUX_HLLC = 2, FLUX_ROE = 3, FLUX_EC = 4, FLUX_GODUNOV = 5,
       FLUX_EC4 = 6 };
// REC_CELLS4 is internal to the kernels: a face reads the four cell values i-1..i+2 with no
// reconstruction (the fourth-order entropy-conservative flux); callers select it as REC_FIRST.
enum { REC_FIRST = 0, REC_MUSCL = 1, REC_WENO3 = 2, REC_ENO2 = 3, REC_CELLS4 = 4 };
enum { BC_PERIODIC = 0, BC_TRANSMISSIVE = 1 };

// Status codes written into the per-sample error words (same values as fv_status).
enum { ST_OK = 0, ST_ENONPHYS = 5, ST_EMAXSTEPS = 6, ST_ECFL = 7 };

constexpr int kThreads = 256;   // threads per workgroup of every stencil kernel

// Physical and grid constants every stencil kernel needs.
struct Phys {
    double gamma;
    double gm1;          // gamma - 1.0, computed at run time
    double vel[3];       // advection velocity
    double inv_dx[3];    // n_k / (hi_k - lo_k)
    double grav;         // shallow water: g
};

// One group of samples on one grid (a batched launch covers one or more groups).
struct Group {
    const double* src;         // U^(s-1): [batch][NF][cells]
    const double* un;          // U^n (read only when use_un != 0)
    double* dst;               // U^(s)
    const double* dt;          // [batch] step size of each sample
    const int32_t* active;     // [batch] nonzero: sample takes this step
    unsigned long long* mbits; // [batch] max wave speed (bit pattern of a double >= 0)
    int32_t* bad;              // [batch] nonzero: a non-physical value was seen
    int64_t cells;             // n0 * n1 * n2
    int32_t n[3];
    int32_t tiles[3];          // tiles per axis
    int32_t ntiles;            // tiles[0] * tiles[1] * tiles[2]
    int32_t batch;
    int64_t block0;            // first block of this group in a multi-group launch
    Phys ph;
    // Split-buffer subdomains (the halo-layout kernels only): the array holds the owned cells
    // n[k] at offset off[k] inside an extent pn[k] per axis (cells = pn[0] pn[1] pn[2]); on the
    // axes of hmask (bit k) the ghost layers are stored in the array, filled by a halo
    // exchange, instead of wrapped. The launch covers the tiles tlo[k] + [0, tcnt[k]).
    int32_t pn[3];
    int32_t off[3];
    int32_t hmask;
    int32_t tlo[3];
    int32_t tcnt[3];
};

constexpr int kMaxGroups = 8;

// The maximum wave speed of a sample is merged into kSpeedSlots words (a workgroup uses slot
// tile % kSpeedSlots), laid out [slot][batch rounded up to 16], so the atomics of one
// sample's workgroups spread over 16 cache lines instead of contending for one word; the
// step control takes the maximum of the slots.
constexpr int kSpeedSlots = 16;
__host__ __device__ inline int64_t speed_pitch(int64_t batch) { return (batch + 15) / 16 * 16; }

// Arguments of one Runge--Kutta stage launch.
struct StageArgs {
    Group g[kMaxGroups];
    int32_t ngroups;
    int32_t bc[3];
    double beta;          // stage weight
    int32_t use_un;       // read U^n from memory (stages >= 2); else U^n == U^(s-1)
    int32_t last;         // last stage: reduce the wave speed and check the new state
    int64_t nblocks;      // total blocks of the launch
};

// Arguments of the wave-speed reduction over a state (no update).
struct SpeedArgs {
    Group g[kMaxGroups];
    int32_t ngroups;
    int64_t nblocks;
};

// Host-side launchers for one (dim, equation, reconstruction, flux, tile) combination.
struct StageKernel {
    void (*stage)(const StageArgs&, hipStream_t);
    void (*speed)(const SpeedArgs&, hipStream_t);
    int32_t bx, by, bz;       // tile shape in cells
    int32_t cells_per_block;  // cells the speed kernel covers per block
};

// Registry (filled by the instantiation units).
const StageKernel* find_stage_kernel(int dim, int eq, int recon, int flux, int variant);
int num_stage_variants(int dim, int eq, int recon, int flux);

}  // namespace fvk
