// 1D Euler: every reconstruction x flux, one row tile of 256 cells.
#include "fv_registry.h"
#include "fv_stage.h"

namespace fvk {
static const RegEntry kTable[] = {
    FV_ALL_RF(1, EQ_EULER, 255, 1, 1, 256),
    FV_ENTRY(1, EQ_EULER, REC_FIRST, FLUX_HLLC, 255, 1, 1, 256),
    FV_ENTRY(1, EQ_EULER, REC_MUSCL, FLUX_HLLC, 255, 1, 1, 256),
    FV_ENTRY(1, EQ_EULER, REC_WENO3, FLUX_HLLC, 255, 1, 1, 256),
};
const RegEntry* unit_euler1d(int* count) { *count = sizeof(kTable) / sizeof(kTable[0]); return kTable; }
}  // namespace fvk
