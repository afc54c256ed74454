// Godunov's flux (the exact Riemann solution at the face) with every reconstruction, for the
// Euler, Burgers and advection equations in 1D, 2D and 3D.
#include "fv_registry.h"
#include "fv_stage.h"

namespace fvk {
#define GOD4(D, E, BX, BY, BZ) FV_ENTRY(D, E, REC_FIRST, FLUX_GODUNOV, BX, BY, BZ, 256), \
    FV_ENTRY(D, E, REC_MUSCL, FLUX_GODUNOV, BX, BY, BZ, 256), FV_ENTRY(D, E, REC_WENO3, FLUX_GODUNOV, BX, BY, BZ, 256), \
    FV_ENTRY(D, E, REC_ENO2, FLUX_GODUNOV, BX, BY, BZ, 256)
#define GOD3(D, BX, BY, BZ) GOD4(D, EQ_EULER, BX, BY, BZ), GOD4(D, EQ_BURGERS, BX, BY, BZ), \
    GOD4(D, EQ_ADVECTION, BX, BY, BZ)
static const RegEntry kTable[] = {GOD3(1, 255, 1, 1), GOD3(2, 16, 15, 1), GOD3(3, 6, 6, 6)};
#undef GOD3
#undef GOD4
const RegEntry* unit_godunov(int* count) { *count = sizeof(kTable) / sizeof(kTable[0]); return kTable; }
}  // namespace fvk
