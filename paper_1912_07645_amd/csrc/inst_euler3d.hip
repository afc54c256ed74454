// 3D Euler: every reconstruction x flux except WENO3 + HLLC (see inst_euler3d_hot.hip).
#include "fv_registry.h"
#include "fv_stage.h"

namespace fvk {
static const RegEntry kTable[] = {
    FV_ALL_RF(3, EQ_EULER, 6, 6, 6, 256),
    FV_ENTRY(3, EQ_EULER, REC_FIRST, FLUX_HLLC, 6, 6, 6, 256),
    FV_ENTRY(3, EQ_EULER, REC_MUSCL, FLUX_HLLC, 6, 6, 6, 256),
};
const RegEntry* unit_euler3d(int* count) { *count = sizeof(kTable) / sizeof(kTable[0]); return kTable; }
}  // namespace fvk
