// Variant table of the batched COCG kernel: every (precision, columns per thread C,
// z-planes per step Z, launch-bound bucket, whole plane or row slabs) instance, for shape
// selection at run time.
#pragma once

#include "cocg_kernel.h"

namespace rpa {
namespace cocg {

using KernelFn = void (*)(Args);

struct Variant {
    int C, Z, bsmax, occ;
    bool slab;           // marches the plane in row slabs (a.nslab >= 2)
    KernelFn f64_real;   // FP64 path, real part of the solution stored
    KernelFn f64_cplx;   // FP64 path, complex solution stored
    KernelFn mixed;      // complex64 state with float64 reliable updates (null if absent)
};

// Defined in cocg_f64.hip and cocg_mixed.hip.
const Variant* f64_variants(int* count);
KernelFn mixed_variant(int C, int Z, int bsmax, int occ, bool slab);

}  // namespace cocg
}  // namespace rpa
