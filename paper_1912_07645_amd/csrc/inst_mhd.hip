// Ideal MHD with the Rusanov and HLL fluxes and every reconstruction, in 1D, 2D and 3D.
#include "fv_registry.h"
#include "fv_stage.h"

namespace fvk {
#define MHD2(D, R, X, Y, Z) FV_ENTRY(D, EQ_MHD, R, FLUX_RUSANOV, X, Y, Z, 256), \
                            FV_ENTRY(D, EQ_MHD, R, FLUX_HLL, X, Y, Z, 256)
#define MHD8(D, X, Y, Z) MHD2(D, REC_FIRST, X, Y, Z), MHD2(D, REC_MUSCL, X, Y, Z), \
                         MHD2(D, REC_WENO3, X, Y, Z), MHD2(D, REC_ENO2, X, Y, Z)
static const RegEntry kTable[] = {MHD8(1, 255, 1, 1), MHD8(2, 16, 15, 1), MHD8(3, 6, 6, 6)};
#undef MHD8
#undef MHD2
const RegEntry* unit_mhd(int* count) { *count = sizeof(kTable) / sizeof(kTable[0]); return kTable; }
}  // namespace fvk
