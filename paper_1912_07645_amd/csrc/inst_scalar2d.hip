// 2D scalar equations (linear advection, Burgers): every reconstruction x (Rusanov, HLL).
#include "fv_registry.h"
#include "fv_stage.h"

namespace fvk {
static const RegEntry kTable[] = {
    FV_ALL_RF(2, EQ_ADVECTION, 16, 15, 1, 256),
    FV_ALL_RF(2, EQ_BURGERS, 16, 15, 1, 256),
};
const RegEntry* unit_scalar2d(int* count) { *count = sizeof(kTable) / sizeof(kTable[0]); return kTable; }
}  // namespace fvk
