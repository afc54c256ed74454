// Shallow-water equations, 1D and 2D: every reconstruction with the Rusanov, HLL and Roe
// fluxes.
#include "fv_registry.h"
#include "fv_stage.h"

namespace fvk {
#define SWE3(D, R, X, Y) FV_ENTRY(D, EQ_SWE, R, FLUX_RUSANOV, X, Y, 1, 256), \
                         FV_ENTRY(D, EQ_SWE, R, FLUX_HLL, X, Y, 1, 256),     \
                         FV_ENTRY(D, EQ_SWE, R, FLUX_ROE, X, Y, 1, 256)
static const RegEntry kTable[] = {
    SWE3(1, REC_FIRST, 255, 1), SWE3(1, REC_MUSCL, 255, 1), SWE3(1, REC_WENO3, 255, 1), SWE3(1, REC_ENO2, 255, 1),
    SWE3(2, REC_FIRST, 16, 15), SWE3(2, REC_MUSCL, 16, 15), SWE3(2, REC_WENO3, 16, 15), SWE3(2, REC_ENO2, 16, 15),
};
#undef SWE3
const RegEntry* unit_swe(int* count) { *count = sizeof(kTable) / sizeof(kTable[0]); return kTable; }
}  // namespace fvk
