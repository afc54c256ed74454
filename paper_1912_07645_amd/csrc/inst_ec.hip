// Entropy-conservative fluxes: Chandrashekar's two-point flux for the Euler equations with
// every reconstruction, and the fourth-order combination for Burgers and Euler, in 1D, 2D
// and 3D. The fourth-order flux is looked up as (REC_FIRST, FLUX_EC4) -- it reads the cell
// values themselves -- and is built with the internal REC_CELLS4 (two ghost layers).
#include "fv_registry.h"
#include "fv_stage.h"

namespace fvk {
#define EC2(D, BX, BY, BZ) FV_ENTRY(D, EQ_EULER, REC_FIRST, FLUX_EC, BX, BY, BZ, 256), \
    FV_ENTRY(D, EQ_EULER, REC_MUSCL, FLUX_EC, BX, BY, BZ, 256), FV_ENTRY(D, EQ_EULER, REC_WENO3, FLUX_EC, BX, BY, BZ, 256), \
    FV_ENTRY(D, EQ_EULER, REC_ENO2, FLUX_EC, BX, BY, BZ, 256)
#define EC4(D, E, BX, BY, BZ) RegEntry{D, E, REC_FIRST, FLUX_EC4, make_stage_kernel<D, E, REC_CELLS4, FLUX_EC4, BX, BY, BZ, 256>()}
static const RegEntry kTable[] = {
    EC2(1, 255, 1, 1), EC2(2, 16, 15, 1), EC2(3, 6, 6, 6),
    EC4(1, EQ_EULER, 255, 1, 1), EC4(2, EQ_EULER, 16, 15, 1), EC4(3, EQ_EULER, 6, 6, 6),
    EC4(1, EQ_BURGERS, 255, 1, 1), EC4(2, EQ_BURGERS, 16, 15, 1), EC4(3, EQ_BURGERS, 6, 6, 6),
};
#undef EC2
#undef EC4
const RegEntry* unit_ec(int* count) { *count = sizeof(kTable) / sizeof(kTable[0]); return kTable; }
}  // namespace fvk
