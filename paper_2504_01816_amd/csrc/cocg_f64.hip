// FP64 instantiations of the batched COCG kernel (see cocg_kernel.h).
#include "cocg_variants.h"

namespace rpa {
namespace cocg {

#define RPA_V(CC, ZZ, BM, OC)                                                            \
    {CC, ZZ, BM, OC, cocg_wg<double, double, CC, ZZ, BM, OC>,                             \
     cocg_wg<double, double2, CC, ZZ, BM, OC>, nullptr}
#define RPA_VZ(CC, ZZ) RPA_V(CC, ZZ, 512, 0), RPA_V(CC, ZZ, 768, 0), RPA_V(CC, ZZ, 1024, 0)
static const Variant kTable[] = {RPA_VZ(1, 1), RPA_VZ(1, 2), RPA_VZ(1, 4),
                                 RPA_VZ(2, 1), RPA_VZ(2, 2), RPA_VZ(2, 4),
                                 RPA_VZ(3, 1), RPA_VZ(3, 2)};
#undef RPA_VZ
#undef RPA_V

const Variant* f64_variants(int* count) {
    *count = int(sizeof(kTable) / sizeof(kTable[0]));
    return kTable;
}

}  // namespace cocg
}  // namespace rpa
