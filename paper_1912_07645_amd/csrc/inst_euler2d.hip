// 2D Euler: every reconstruction x flux except WENO3 + HLLC (see inst_euler2d_hot.hip).
// MUSCL + HLL (the multilevel configuration) and MUSCL + Rusanov (the adjoint configuration)
// also have the unheld form, whose stage prefetches U^n, for the tuner.
#include "fv_registry.h"
#include "fv_stage.h"

namespace fvk {
static const RegEntry kTable[] = {
    FV_ALL_RF(2, EQ_EULER, 16, 15, 1, 256),
    FV_ENTRY(2, EQ_EULER, REC_FIRST, FLUX_HLLC, 16, 15, 1, 256),
    FV_ENTRY(2, EQ_EULER, REC_MUSCL, FLUX_HLLC, 16, 15, 1, 256),
    FV_ENTRY_H(2, EQ_EULER, REC_MUSCL, FLUX_HLL, 16, 15, 1, 256, 0),
    FV_ENTRY_H(2, EQ_EULER, REC_MUSCL, FLUX_RUSANOV, 16, 15, 1, 256, 0),
};
const RegEntry* unit_euler2d(int* count) { *count = sizeof(kTable) / sizeof(kTable[0]); return kTable; }
}  // namespace fvk
