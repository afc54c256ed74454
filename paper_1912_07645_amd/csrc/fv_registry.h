// fv_registry.h -- registration of the stencil kernel instantiations.
#pragma once

#include "fv_common.h"

namespace fvk {

struct RegEntry {
    int dim, eq, recon, flux;
    StageKernel k;
};

// Each instantiation unit exposes its table through one of these functions.
#define FV_DECLARE_UNIT(name) \
    const RegEntry* name(int* count);

FV_DECLARE_UNIT(unit_euler1d)
FV_DECLARE_UNIT(unit_euler2d)
FV_DECLARE_UNIT(unit_euler2d_hot)
FV_DECLARE_UNIT(unit_euler3d)
FV_DECLARE_UNIT(unit_euler3d_hot)
FV_DECLARE_UNIT(unit_scalar1d)
FV_DECLARE_UNIT(unit_scalar2d)
FV_DECLARE_UNIT(unit_scalar3d)
FV_DECLARE_UNIT(unit_more1d)
FV_DECLARE_UNIT(unit_more2d)
FV_DECLARE_UNIT(unit_more3d)
FV_DECLARE_UNIT(unit_godunov)
FV_DECLARE_UNIT(unit_ec)
FV_DECLARE_UNIT(unit_mhd)
FV_DECLARE_UNIT(unit_swe)

}  // namespace fvk

// Helpers for the instantiation units.
#define FV_ENTRY(D, E, R, F, X, Y, Z, NT) \
    RegEntry{D, E, R, F, make_stage_kernel<D, E, R, F, X, Y, Z, NT>()}
#define FV_ENTRY_H(D, E, R, F, X, Y, Z, NT, H) \
    RegEntry{D, E, R, F, make_stage_kernel<D, E, R, F, X, Y, Z, NT, H>()}

#define FV_ENTRY_Z(E, R, F, X, Y, Z, NT, WPE) \
    RegEntry{3, E, R, F, make_stage_kernel_z<E, R, F, X, Y, Z, NT, WPE>()}

#define FV_ALL_RF(D, E, X, Y, Z, NT)                                                          \
    FV_ENTRY(D, E, REC_FIRST, FLUX_RUSANOV, X, Y, Z, NT), FV_ENTRY(D, E, REC_FIRST, FLUX_HLL, X, Y, Z, NT), \
    FV_ENTRY(D, E, REC_MUSCL, FLUX_RUSANOV, X, Y, Z, NT), FV_ENTRY(D, E, REC_MUSCL, FLUX_HLL, X, Y, Z, NT), \
    FV_ENTRY(D, E, REC_WENO3, FLUX_RUSANOV, X, Y, Z, NT), FV_ENTRY(D, E, REC_WENO3, FLUX_HLL, X, Y, Z, NT)
