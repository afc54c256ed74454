// 3D Euler WENO3 + HLLC: tile shapes for the tuner (6x6x6: 756 faces for 3 x 256 lanes;
// 8x6x6: 996 faces for 4 x 256 lanes).
#include "fv_registry.h"
#include "fv_stage.h"

namespace fvk {
static const RegEntry kTable[] = {
    FV_ENTRY(3, EQ_EULER, REC_WENO3, FLUX_HLLC, 6, 6, 6, 256),
    FV_ENTRY(3, EQ_EULER, REC_WENO3, FLUX_HLLC, 8, 6, 6, 256),
    FV_ENTRY(3, EQ_EULER, REC_WENO3, FLUX_HLLC, 8, 4, 4, 256),
};
const RegEntry* unit_euler3d_hot(int* count) { *count = sizeof(kTable) / sizeof(kTable[0]); return kTable; }
}  // namespace fvk
