// 2D Euler WENO3 + HLLC (the Kelvin--Helmholtz configuration): tile shapes for the tuner.
// Each shape's face list, padded per axis to whole wavefronts, fills whole passes:
// 16x15: 256 + 256 for 2 x 256 lanes, 32x15 on 512 threads: 512 + 512, 32x7: 256 + 256,
// 16x13: 256 + 256 (5056 tiles at 1024^2, a whole number of rounds of resident workgroups).
// Fluxes are held in registers (LDS = max(tile, faces)) except for the second entry.
#include "fv_registry.h"
#include "fv_stage.h"

namespace fvk {
static const RegEntry kTable[] = {
    FV_ENTRY(2, EQ_EULER, REC_WENO3, FLUX_HLLC, 16, 15, 1, 256),
    FV_ENTRY_H(2, EQ_EULER, REC_WENO3, FLUX_HLLC, 16, 15, 1, 256, 0),
    FV_ENTRY(2, EQ_EULER, REC_WENO3, FLUX_HLLC, 32, 15, 1, 512),
    FV_ENTRY(2, EQ_EULER, REC_WENO3, FLUX_HLLC, 32, 7, 1, 256),
    FV_ENTRY(2, EQ_EULER, REC_WENO3, FLUX_HLLC, 16, 13, 1, 256),
};
const RegEntry* unit_euler2d_hot(int* count) { *count = sizeof(kTable) / sizeof(kTable[0]); return kTable; }
}  // namespace fvk
