// FP64 instantiations of the batched COCG kernel (see cocg_kernel.h).
#include "cocg_variants.h"

namespace rpa {
namespace cocg {

#define RPA_V(CC, ZZ, BM, OC, SL)                                                        \
    {CC, ZZ, BM, OC, SL, cocg_wg<double, double, CC, ZZ, BM, OC, SL>,                     \
     cocg_wg<double, double2, CC, ZZ, BM, OC, SL>, nullptr}
#define RPA_VZ(CC, ZZ) \
    RPA_V(CC, ZZ, 512, 0, false), RPA_V(CC, ZZ, 768, 0, false), RPA_V(CC, ZZ, 1024, 0, false)
#define RPA_VS(ZZ) \
    RPA_V(1, ZZ, 512, 0, true), RPA_V(1, ZZ, 768, 0, true), RPA_V(1, ZZ, 1024, 0, true)
static const Variant kTable[] = {RPA_VZ(1, 1), RPA_VZ(1, 2), RPA_VZ(1, 4),
                                 RPA_VZ(2, 1), RPA_VZ(2, 2), RPA_VZ(2, 4),
                                 RPA_VZ(3, 1), RPA_VZ(3, 2),
                                 RPA_VS(1),    RPA_VS(2)};
#undef RPA_VS
#undef RPA_VZ
#undef RPA_V

const Variant* f64_variants(int* count) {
    *count = int(sizeof(kTable) / sizeof(kTable[0]));
    return kTable;
}

}  // namespace cocg
}  // namespace rpa
