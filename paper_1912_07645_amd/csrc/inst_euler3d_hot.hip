// 3D Euler WENO3 + HLLC: tile shapes for the tuner (6x6x6: 3 x 256 padded faces for
// 3 x 256 lanes; 8x8x4: 3 x 320 for 4 x 256 lanes).
#include "fv_registry.h"
#include "fv_stage.h"

namespace fvk {
static const RegEntry kTable[] = {
    FV_ENTRY(3, EQ_EULER, REC_WENO3, FLUX_HLLC, 6, 6, 6, 256),
    FV_ENTRY(3, EQ_EULER, REC_WENO3, FLUX_HLLC, 8, 8, 4, 256),
};
const RegEntry* unit_euler3d_hot(int* count) { *count = sizeof(kTable) / sizeof(kTable[0]); return kTable; }
}  // namespace fvk
