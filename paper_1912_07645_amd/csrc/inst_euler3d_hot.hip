// 3D Euler WENO3 + HLLC: tile shapes for the tuner. Cube tiles: 6x6x6 (3 x 256 padded faces
// for 3 x 256 lanes), 8x8x4 (3 x 320 for 4 x 256 lanes). z-marching column blocks: 16x15
// (255 + 256 plane faces, 240 columns) and 32x7 (231 + 256, 224 columns) over 32 or 64 planes,
// compiled for 3 wavefronts per SIMD, and 16x15 also for 4.
#include "fv_registry.h"
#include "fv_stage.h"
#include "fv_stage_z.h"

namespace fvk {
static const RegEntry kTable[] = {
    FV_ENTRY(3, EQ_EULER, REC_WENO3, FLUX_HLLC, 6, 6, 6, 256),
    FV_ENTRY(3, EQ_EULER, REC_WENO3, FLUX_HLLC, 8, 8, 4, 256),
    FV_ENTRY_Z(EQ_EULER, REC_WENO3, FLUX_HLLC, 16, 15, 32, 256, 3),
    FV_ENTRY_Z(EQ_EULER, REC_WENO3, FLUX_HLLC, 16, 15, 64, 256, 3),
    FV_ENTRY_Z(EQ_EULER, REC_WENO3, FLUX_HLLC, 32, 7, 32, 256, 3),
    FV_ENTRY_Z(EQ_EULER, REC_WENO3, FLUX_HLLC, 16, 15, 32, 256, 4),
};
const RegEntry* unit_euler3d_hot(int* count) { *count = sizeof(kTable) / sizeof(kTable[0]); return kTable; }
}  // namespace fvk
