// Launch-shape selection for the batched COCG kernel (design in cocg_kernel.h).
//
// A shape is (C columns per thread, Z z-planes per barrier step, block size, launch-bound
// bucket, row slabs per plane).  Candidates are the compiled variants; each one's register
// count and scratch (spill) size are read from the runtime, and the choice is the spill-free
// variant that leaves the fewest idle columns, then the one with more planes per step (when
// every variant spills, the one that spills least).  Large
// planes whose whole-plane variants all spill are marched in row slabs (one column per
// thread, at least 12 rows per slab, whose 12 halo rows are re-read from memory per sweep).
// A shape measured by the autotuner for the same precision and grid (tuning file) takes
// precedence, and RPA_COCG_SHAPE="C,Z,bsmax[,bs[,occ[,nslab]]]" forces one (used by the
// autotuner itself).  A forced shape that is not valid for the grid falls back to the
// automatic choice.  RPA_COCG_VERBOSE=1 prints the chosen shape of every launch to stderr.
// RPA_MIXED_BD_TOL replaces the complex64 kernel's breakdown threshold (1e-10; tests raise it to
// force breakdowns and exercise the FP64 restart).
#include <dlfcn.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "cocg_variants.h"

namespace rpa {

namespace {

// Tuned shapes from the autotuner: lines "precision n0 n1 n2 C Z bsmax bs occ [nslab]", read
// once from RPA_TUNE_FILE or from cocg_shapes.txt next to this shared library.
struct Tuned {
    bool mixed;
    int n0, n1, n2, C, Z, bsmax, bs, occ, nslab;
};

const std::vector<Tuned>& tuned_shapes() {
    static std::vector<Tuned> table;
    static std::once_flag once;
    std::call_once(once, [] {
        std::string path;
        if (const char* env = std::getenv("RPA_TUNE_FILE")) {
            path = env;
        } else {
            Dl_info info{};
            if (dladdr(reinterpret_cast<void*>(&tuned_shapes), &info) && info.dli_fname) {
                path = info.dli_fname;
                const size_t cut = path.find_last_of('/');
                path = (cut == std::string::npos ? std::string(".") : path.substr(0, cut)) +
                       "/cocg_shapes.txt";
            }
        }
        FILE* f = path.empty() ? nullptr : std::fopen(path.c_str(), "r");
        if (!f) return;
        char line[256], prec[16];
        while (std::fgets(line, sizeof line, f)) {
            Tuned t{};
            t.nslab = 1;
            if (std::sscanf(line, "%15s %d %d %d %d %d %d %d %d %d", prec, &t.n0, &t.n1, &t.n2,
                            &t.C, &t.Z, &t.bsmax, &t.bs, &t.occ, &t.nslab) < 9)
                continue;
            t.mixed = std::strcmp(prec, "mixed") == 0;
            table.push_back(t);
        }
        std::fclose(f);
    });
    return table;
}

struct Chosen {
    cocg::KernelFn fn = nullptr;
    int C = 0, Z = 0, bs = 0, nbuf = 2, nslab = 1, rows = 0;
    size_t lds = 0;
};

// Reduction scratch plus nbuf buffers of Z staged planes (rows of the slab, 6 ghost columns
// and 6 ghost rows on each side).  Elements are 16 B (the FP64 queue entry, also used by the
// true-residual sweep of the mixed kernel).
int lds_row(int n0) { return (n0 + 12 + 7) / 8 * 8; }

size_t lds_bytes(int n0, int rows, int Z, int nbuf) {
    const size_t pl = size_t(rows + 12) * size_t(lds_row(n0));
    return 16 * 8 * sizeof(double) + size_t(nbuf) * size_t(Z) * pl * 16;
}

bool attrs(cocg::KernelFn fn, int* regs, size_t* scratch) {
    hipFuncAttributes at{};
    if (hipFuncGetAttributes(&at, reinterpret_cast<const void*>(fn)) != hipSuccess) return false;
    *regs = at.numRegs;
    *scratch = at.localSizeBytes;
    return true;
}

Chosen choose(const Grid& g, bool mixed, bool xcomplex, bool allow_forced) {
    const int P = g.n0 * g.n1;
    int nv = 0;
    const cocg::Variant* tab = cocg::f64_variants(&nv);
    int fC = 0, fZ = 0, fB = 0, fBS = 0, fO = 0, fS = 0;
    if (!allow_forced) {
        // automatic choice only
    } else if (const char* env = std::getenv("RPA_COCG_SHAPE")) {
        if (std::sscanf(env, "%d,%d,%d,%d,%d,%d", &fC, &fZ, &fB, &fBS, &fO, &fS) < 3)
            fC = fZ = fB = fBS = fO = fS = 0;
    } else {
        for (const Tuned& t : tuned_shapes())
            if (t.mixed == mixed && t.n0 == g.n0 && t.n1 == g.n1 && t.n2 == g.n2) {
                fC = t.C;
                fZ = t.Z;
                fB = t.bsmax;
                fBS = t.bs;
                fO = t.occ;
                fS = t.nslab;
            }
    }
    Chosen best;
    double best_cost = 1e30;
    for (int k = 0; k < nv; ++k) {
        const cocg::Variant& v = tab[k];
        cocg::KernelFn fn = mixed ? cocg::mixed_variant(v.C, v.Z, v.bsmax, v.occ, v.slab)
                                  : (xcomplex ? v.f64_cplx : v.f64_real);
        if (!fn) continue;
        if (g.n2 % v.Z != 0) continue;
        int regs = 0;
        size_t scratch = 0;
        if (!attrs(fn, &regs, &scratch)) continue;
        if (fC && (v.C != fC || v.Z != fZ || v.bsmax != fB || v.occ != fO)) continue;
        if (!fC && v.occ != 0) continue;          // capped variants only when tuned or forced
        // whole plane: one slab; slab variants: 2 .. n1/12 slabs of equal height
        const int s_lo = v.slab ? 2 : 1, s_hi = v.slab ? g.n1 / 12 : 1;
        for (int nslab = s_lo; nslab <= s_hi; ++nslab) {
            if (g.n1 % nslab != 0) continue;
            if (fC && (fS > 1 ? fS : 1) != nslab) continue;
            const int rows = g.n1 / nslab;
            const int ps = rows * g.n0;               // columns per slab
            int bs = ((ps + v.C - 1) / v.C + 63) / 64 * 64;
            if (fBS && fBS >= bs && fBS % 64 == 0) bs = fBS;   // forced wider block (idle lanes)
            if (bs > v.bsmax) continue;
            const int lower = v.bsmax == 512 ? 0 : v.bsmax == 768 ? 512 : 768;
            if (bs <= lower) continue;                       // use the tightest bucket
            if (v.slab && 12 * g.n0 > bs) continue;          // one halo entry per thread
            int nbuf = 2;
            size_t lds = lds_bytes(g.n0, rows, v.Z, 2);
            if (lds > 150 * 1024) {
                nbuf = 1;
                lds = lds_bytes(g.n0, rows, v.Z, 1);
            }
            if (lds > 150 * 1024) continue;
            const double idle = double(bs * v.C - ps) / double(bs * v.C);
            // halo rows re-read per slab: 12 / rows extra reads of the swept vector
            const double halo = v.slab ? 12.0 / rows : 0.0;
            // spills, by spilled bytes per lane: a few dozen spilled registers cost less than
            // the halo re-reads of a slab split (measured at 28^3 and 32^3), hundreds far more
            const double spill = double(scratch) / 256.0;
            double cost = idle + halo + spill + 0.03 * (4 - v.Z) + 0.05 * (2 - nbuf);
            if (cost < best_cost - 1e-12) {
                best_cost = cost;
                best = Chosen{fn, v.C, v.Z, bs, nbuf, nslab, rows, lds};
            }
        }
    }
    return best;
}

// The geometric part of choose(): some compiled variant fits the grid's plane (block size,
// slab height, halo threads, LDS), whatever its register use.
bool geometry_fits(const Grid& g, const cocg::Variant& v) {
    if (g.n2 % v.Z != 0) return false;
    const int s_lo = v.slab ? 2 : 1, s_hi = v.slab ? g.n1 / 12 : 1;
    for (int nslab = s_lo; nslab <= s_hi; ++nslab) {
        if (g.n1 % nslab != 0) continue;
        const int rows = g.n1 / nslab;
        const int ps = rows * g.n0;
        const int bs = ((ps + v.C - 1) / v.C + 63) / 64 * 64;
        if (bs > v.bsmax) continue;
        if (v.slab && 12 * g.n0 > bs) continue;
        if (lds_bytes(g.n0, rows, v.Z, 1) > 150 * 1024) continue;
        return true;
    }
    return false;
}

}  // namespace

bool cocg_shape_exists(const Grid& g, bool mixed) {
    int nv = 0;
    const cocg::Variant* tab = cocg::f64_variants(&nv);
    bool f64 = false, mx = !mixed;
    for (int k = 0; k < nv; ++k) {
        const cocg::Variant& v = tab[k];
        if (v.occ != 0 || !geometry_fits(g, v)) continue;
        f64 = true;
        if (mixed && cocg::mixed_variant(v.C, v.Z, v.bsmax, v.occ, v.slab)) mx = true;
    }
    return f64 && mx;
}

hipError_t launch_cocg(const CocgLaunch& L, hipStream_t s) {
    if (L.nsys <= 0) return hipSuccess;
    cocg::Args a{};
    a.n0 = L.g.n0;
    a.n1 = L.g.n1;
    a.n2 = L.g.n2;
    a.P = L.g.n0 * L.g.n1;
    double w[7];
    fd_weights(w);
    const double ih2 = 1.0 / (L.g.h * L.g.h);
    a.cw[0] = -0.5 * 3.0 * w[0] * ih2;
    for (int k = 1; k <= 6; ++k) a.cw[k] = -0.5 * w[k] * ih2;
    a.vloc = L.vloc;
    a.eps = L.eps;
    a.ns = L.ns;
    a.omega = L.omega;
    a.omega_v = L.omega_v;
    a.order = L.order;
    a.tol2 = L.tol * L.tol;
    a.refine2 = L.refine_tol * L.refine_tol;
    a.refine_gap = L.refine_gap;
    a.vloc32 = L.vloc32;
    a.max_iter = L.max_iter;
    a.bd_tol = L.fp32 ? 1e-10 : 1e-14;
    if (L.fp32)
        if (const char* e = std::getenv("RPA_MIXED_BD_TOL")) a.bd_tol = std::atof(e);
    a.nd = L.g.nd();
    a.r = L.r;
    a.pa = L.pa;
    a.pb = L.pb;
    a.x = L.x;
    a.xlo = L.xlo;
    a.rhi = L.rhi;
    a.iters = L.iters;
    a.status = L.status;
    a.refinements = L.refinements;
    a.b2 = L.b2;
    a.x_accum = L.x_accum ? 1 : 0;
    Chosen ch = choose(L.g, L.fp32, L.x_complex, true);
    if (!ch.fn) ch = choose(L.g, L.fp32, L.x_complex, false);
    if (!ch.fn) return hipErrorInvalidConfiguration;
    a.nbuf = ch.nbuf;
    a.rs = lds_row(L.g.n0);
    a.nslab = ch.nslab;
    a.rows = ch.rows;
    a.periodic = L.g.periodic() ? 1 : 0;
    if (std::getenv("RPA_COCG_VERBOSE"))
        std::fprintf(stderr, "cocg shape C=%d Z=%d bs=%d nbuf=%d nslab=%d rows=%d lds=%zu\n",
                     ch.C, ch.Z, ch.bs, ch.nbuf, ch.nslab, ch.rows, ch.lds);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(ch.fn),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(ch.lds));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(ch.fn, dim3(L.nsys), dim3(ch.bs), ch.lds, s, a);
    return hipGetLastError();
}

}  // namespace rpa
