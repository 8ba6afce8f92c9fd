// Mixed-precision instantiations of the batched COCG kernel (complex64 state, float64
// reliable updates; see cocg_kernel.h).
#include "cocg_variants.h"

namespace rpa {
namespace cocg {

KernelFn mixed_variant(int C, int Z, int bsmax, int occ, bool slab) {
#define RPA_CASE(CC, ZZ, BM, OC, SL)                                              \
    if (C == CC && Z == ZZ && bsmax == BM && occ == OC && slab == SL)             \
        return cocg_wg<float, float2, CC, ZZ, BM, OC, SL>;
#define RPA_CZ(CC, ZZ) \
    RPA_CASE(CC, ZZ, 512, 0, false) RPA_CASE(CC, ZZ, 768, 0, false) RPA_CASE(CC, ZZ, 1024, 0, false)
    RPA_CZ(1, 1) RPA_CZ(1, 2) RPA_CZ(1, 4) RPA_CZ(2, 1) RPA_CZ(2, 2) RPA_CZ(2, 4)
    RPA_CZ(3, 1) RPA_CZ(3, 2)
    RPA_CASE(1, 1, 512, 0, true) RPA_CASE(1, 1, 768, 0, true) RPA_CASE(1, 1, 1024, 0, true)
    RPA_CASE(1, 2, 512, 0, true) RPA_CASE(1, 2, 768, 0, true) RPA_CASE(1, 2, 1024, 0, true)
#undef RPA_CZ
#undef RPA_CASE
    return nullptr;
}

}  // namespace cocg
}  // namespace rpa
