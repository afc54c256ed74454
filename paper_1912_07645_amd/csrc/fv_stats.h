// fv_stats.h -- statistics kernels (internal).
#pragma once

#include "fv_common.h"

namespace fvk {

// Fine grid, coarse grid and their integer refinement ratio per axis.
struct DiffGeom {
    int32_t nf[3];
    int32_t nc[3];
    int32_t r[3];
};

constexpr int kMaxLevels = 8;

struct CombineArgs {
    const double* mean[kMaxLevels];  // [quantity][cells of level l]
    int32_t n[kMaxLevels][3];        // grid of level l
    int32_t r[kMaxLevels][3];        // finest / level l, per axis
    int32_t nfine[3];
    int32_t nlevels;
    int32_t nq;
};

void launch_welford_diff(int nf, int kind, const double* fine, const double* coarse,
                         const DiffGeom& geo, int32_t batch, int64_t count0, double* mean,
                         double* m2, hipStream_t s);
void launch_mlmc_combine(const CombineArgs& a, double* out, hipStream_t s);

// Workgroups per (sample, quantity) of the structure-function pass.
int sf_blocks_per_field(int32_t dim, const int32_t n[3], int32_t max_h);
// qout (may be null): also write the quantity fields of the batch, [sample][quantity][cells].
void launch_welford(int nf, int kind, const double* state, int64_t cells, int32_t batch,
                    int64_t count0, double* mean, double* m2, double* qout, hipStream_t s);
// Whether max_h lags run on the staged kernels, which can form the quantities themselves.
bool sf_staged(int32_t max_h);
// kind < 0: q holds the quantities ([sample][quantity][cells]). kind >= 0 (staged kernels
// only): q is the state, and the quantities are formed from it as launch_welford forms them.
void launch_sf_partial(const double* q, int32_t dim, const int32_t n[3], int32_t nq, int32_t max_h,
                       int32_t batch, int kind, double* partial, hipStream_t s);
// x: scratch of batch * nq * max_h doubles (S_q(h) of each sample of the chunk).
void launch_sf_welford(const double* partial, int32_t nq, int32_t max_h, int32_t nblk,
                       int32_t batch, int64_t count0, double denom, double* x, double* s2mean,
                       double* s2m2, hipStream_t s);
void launch_variance(const double* m2, int64_t n, double count, double* var, hipStream_t s);
void launch_fill_zero(double* p, int64_t n, hipStream_t s);

}  // namespace fvk
