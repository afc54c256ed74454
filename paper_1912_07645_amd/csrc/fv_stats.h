// fv_stats.h -- statistics kernels (internal).
#pragma once

#include "fv_common.h"

namespace fvk {

int sf_blocks_per_field(int64_t cells);
void launch_welford(int nf, bool euler, const double* state, int64_t cells, int32_t batch,
                    int64_t count0, double* mean, double* m2, hipStream_t s);
void launch_quantities(int nf, bool euler, const double* state, int64_t cells, int32_t batch,
                       double* q, hipStream_t s);
void launch_sf_partial(const double* q, int32_t dim, const int32_t n[3], int32_t nq, int32_t max_h,
                       int32_t batch, double* partial, hipStream_t s);
void launch_sf_welford(const double* partial, int32_t nq, int32_t max_h, int32_t nblk,
                       int32_t batch, int64_t count0, double denom, double* s2mean, double* s2m2,
                       hipStream_t s);
void launch_variance(const double* m2, int64_t n, double count, double* var, hipStream_t s);
void launch_fill_zero(double* p, int64_t n, hipStream_t s);

}  // namespace fvk
