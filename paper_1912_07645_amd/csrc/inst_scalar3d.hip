// 3D scalar equations (linear advection, Burgers): every reconstruction x (Rusanov, HLL).
#include "fv_registry.h"
#include "fv_stage.h"

namespace fvk {
static const RegEntry kTable[] = {
    FV_ALL_RF(3, EQ_ADVECTION, 6, 6, 6, 256),
    FV_ALL_RF(3, EQ_BURGERS, 6, 6, 6, 256),
};
const RegEntry* unit_scalar3d(int* count) { *count = sizeof(kTable) / sizeof(kTable[0]); return kTable; }
}  // namespace fvk
