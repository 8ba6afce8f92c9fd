// Mixed-precision instantiations of the batched COCG kernel (complex64 state, float64
// reliable updates; see cocg_kernel.h).
#include "cocg_variants.h"

namespace rpa {
namespace cocg {

KernelFn mixed_variant(int C, int Z, int bsmax, int occ) {
#define RPA_CASE(CC, ZZ, BM, OC) \
    if (C == CC && Z == ZZ && bsmax == BM && occ == OC) return cocg_wg<float, float2, CC, ZZ, BM, OC>;
#define RPA_CZ(CC, ZZ) RPA_CASE(CC, ZZ, 512, 0) RPA_CASE(CC, ZZ, 768, 0) RPA_CASE(CC, ZZ, 1024, 0)
    RPA_CZ(1, 1) RPA_CZ(1, 2) RPA_CZ(1, 4) RPA_CZ(2, 1) RPA_CZ(2, 2) RPA_CZ(2, 4)
    RPA_CZ(3, 1) RPA_CZ(3, 2)
#undef RPA_CZ
#undef RPA_CASE
    return nullptr;
}

}  // namespace cocg
}  // namespace rpa
