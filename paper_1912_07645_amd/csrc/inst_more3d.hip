// 3D: the Roe flux with every reconstruction, second-order ENO with every other flux, and
// Tadmor's entropy-conservative flux for Burgers.
#include "fv_registry.h"
#include "fv_stage.h"

namespace fvk {
#define ROE4(E) FV_ENTRY(3, E, REC_FIRST, FLUX_ROE, 6, 6, 6, 256), FV_ENTRY(3, E, REC_MUSCL, FLUX_ROE, 6, 6, 6, 256), \
                FV_ENTRY(3, E, REC_WENO3, FLUX_ROE, 6, 6, 6, 256), FV_ENTRY(3, E, REC_ENO2, FLUX_ROE, 6, 6, 6, 256)
#define ENO2(E, F) FV_ENTRY(3, E, REC_ENO2, F, 6, 6, 6, 256)
static const RegEntry kTable[] = {
    ROE4(EQ_EULER), ENO2(EQ_EULER, FLUX_RUSANOV), ENO2(EQ_EULER, FLUX_HLL), ENO2(EQ_EULER, FLUX_HLLC),
    ROE4(EQ_BURGERS), ENO2(EQ_BURGERS, FLUX_RUSANOV), ENO2(EQ_BURGERS, FLUX_HLL),
    FV_ENTRY(3, EQ_BURGERS, REC_FIRST, FLUX_EC, 6, 6, 6, 256), FV_ENTRY(3, EQ_BURGERS, REC_MUSCL, FLUX_EC, 6, 6, 6, 256),
    FV_ENTRY(3, EQ_BURGERS, REC_WENO3, FLUX_EC, 6, 6, 6, 256), FV_ENTRY(3, EQ_BURGERS, REC_ENO2, FLUX_EC, 6, 6, 6, 256),
    ROE4(EQ_ADVECTION), ENO2(EQ_ADVECTION, FLUX_RUSANOV), ENO2(EQ_ADVECTION, FLUX_HLL),
};
#undef ROE4
#undef ENO2
const RegEntry* unit_more3d(int* count) { *count = sizeof(kTable) / sizeof(kTable[0]); return kTable; }
}  // namespace fvk
