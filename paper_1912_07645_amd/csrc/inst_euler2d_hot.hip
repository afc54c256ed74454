// 2D Euler WENO3 + HLLC (the Kelvin--Helmholtz configuration): tile shapes and LDS plans for
// the tuner. Each shape's face list, padded per axis to whole wavefronts, fills whole passes
// (16x15: 256 + 256 faces for 2 x 256 lanes; 32x15 on 512 threads: 512 + 512).
//   split faces (HOLD = 2): 16x15 on 256 threads, 32x15 on 512 threads;
//   tile and faces side by side in LDS (HOLD = 0): 16x15;
//   fluxes held in registers over the dead tile (HOLD = 1): 16x15.
#include "fv_registry.h"
#include "fv_stage.h"

namespace fvk {
static const RegEntry kTable[] = {
    FV_ENTRY(2, EQ_EULER, REC_WENO3, FLUX_HLLC, 16, 15, 1, 256),
    FV_ENTRY(2, EQ_EULER, REC_WENO3, FLUX_HLLC, 32, 15, 1, 512),
    FV_ENTRY_H(2, EQ_EULER, REC_WENO3, FLUX_HLLC, 16, 15, 1, 256, 0),
    FV_ENTRY_H(2, EQ_EULER, REC_WENO3, FLUX_HLLC, 16, 15, 1, 256, 1),
};
const RegEntry* unit_euler2d_hot(int* count) { *count = sizeof(kTable) / sizeof(kTable[0]); return kTable; }
}  // namespace fvk
