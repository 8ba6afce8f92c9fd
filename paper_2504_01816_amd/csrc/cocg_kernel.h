// Batched COCG kernel for the shifted Sternheimer systems (H - eps_n - i omega) x = b
// (Sec. 3: COCG, conjugate gradients with the unconjugated bilinear form; Eq. 9).
//
// Design (gfx950):
//  * One workgroup owns one system for its whole solve.  The reductions of a COCG
//    iteration are workgroup-local, so a system runs all its iterations inside one launch
//    with no host round trip.  Systems converge independently; a finished workgroup frees
//    its CU slot and the dispatcher starts the next system (active-set compaction).
//  * An iteration is two streaming sweeps over the system:
//      sweep 1: p <- r + beta p (into the other p buffer), q = A p; reduce p^T q, |p|^2, |q|^2
//      sweep 2: q = A p again (q is never stored), x <- x + alpha p, r <- r - alpha q;
//               reduce r^T r, |r|^2.
//  * A sweep marches along z, Z planes per step.  Thread t owns columns t, t+BS, ... of
//    the x-y plane and holds planes z-6 .. z+5+Z of the swept vector in a register queue;
//    the Z current planes are staged in LDS (double buffered) for the x and y neighbours.
//    The next step's planes are loaded before the current step computes, and the barrier
//    only orders LDS (global loads and stores stay in flight): every global address is
//    read and written by one thread only, so LDS is the sole cross-thread channel.
//  * Large planes (whose whole-plane columns per thread would spill registers) are marched
//    in row slabs, one after another, one column per thread: each slab's 6 rows above and
//    below are read from memory for every centre plane, and each sweep ends with a
//    workgroup-wide memory barrier, since the next sweep reads rows that other threads wrote.
//    In sweep 1 of the FP64 kernel the halo rows that belong to a slab marched earlier in the
//    same sweep are read from the p_new that slab wrote (one vector instead of r and p; a
//    memory barrier between slabs); the others are formed from r and p as the slab's own rows
//    are.
//  * Mixed precision (T = float): r, p and the partial solution x_lo are complex64; the
//    solution x_hi and the residual r_hi are complex float64.  When the complex64 residual
//    has dropped by refine_tol since the last update, at least refine_gap iterations after it
//    (or reaches the tolerance, or the cap), a reliable update (group-wise residual
//    replacement) runs: x_hi += x_lo and r_hi -= A x_lo, with
//    A x_lo evaluated in float64 from the exact complex64 values, so r_hi = b - A x_hi holds
//    to float64 rounding; then r <- complex64(r_hi).  p and the Krylov recurrence continue.
//    The tolerance test uses |r_hi|.  A solve that stops at the iteration cap or at a
//    breakdown of the complex64 recurrence ends with a reliable update too, so the host can
//    restart it in FP64 from x_hi and the exact residual.
//  * Reductions accumulate in float64 and are fixed-order: results are bitwise
//    reproducible run to run.
// Layout: state arrays are system-major, nsys x N_d, complex interleaved (re, im).
// Constraints: n2 >= 12 and divisible by Z; n0, n1 >= 7; slab mode: rows >= 12 and at
// least 12 n0 threads.
#pragma once

#include <type_traits>

#include "internal.h"

namespace rpa {
namespace cocg {

template <typename T> struct Cplx;
template <> struct Cplx<double> { using type = double2; };
template <> struct Cplx<float> { using type = float2; };

// Arithmetic precision of the COCG recurrences for a state precision T (reductions always
// accumulate in float64).  The mixed path computes q = A p and the updates in float32 on its
// complex64 state.  Built with RPA_MIXED_ARITH=double it computes them in float64 from the
// stored complex64 values instead, rounding only when it stores: measured on the 48^3 cell,
// that removes about a fifth of the iteration inflation at the lowest frequency (1.70x the
// FP64 iterations against 2.18x) but costs a quarter more time per iteration (conversions and
// register spills of the slab variants), a net loss.
#ifndef RPA_MIXED_ARITH
#define RPA_MIXED_ARITH float
#endif
template <typename T> struct Arith { using type = double; };
template <> struct Arith<float> { using type = RPA_MIXED_ARITH; };

struct Args {
    int n0, n1, n2, P;
    double cw[7];          // cw[k] = -1/2 w_k / h^2 for k >= 1; cw[0] = -1/2 * 3 w_0 / h^2
    const double* vloc;
    const float* vloc32;   // mixed: V_loc rounded to float32, read by the float32 sweeps (half
                           // the bytes; the float32 diagonal rounds anyway); required there
    const double* eps;
    int ns;
    double omega;          // shift of every system when omega_v is null
    const double* omega_v; // per trial vector j (system s = n + ns j): its frequency, or null
    const int* order;      // workgroup b solves system order[b] (a permutation), or null
    double tol2;
    double refine2;        // mixed: refine_tol^2
    int refine_gap;        // mixed: fewest iterations between two reliable updates (except at
                           // the tolerance and the cap)
    int max_iter;
    double bd_tol;
    int64_t nd;
    void* r;               // complex T
    void* pa;              // complex T
    void* pb;              // complex T
    void* x;               // FP64 path: real or complex double; mixed: complex double x_hi
    void* xlo;             // mixed: complex float
    double* rhi;           // mixed: complex double residual (starts at the right-hand side)
    int* iters;
    int* status;
    int* refinements;      // mixed: per system
    int nbuf;              // LDS plane buffers (2: one barrier per step, 1: two barriers)
    int rs;                // LDS row stride in entries: n0 + 12 rounded up to a multiple of 8
    int periodic;          // 1: periodic cell; 0: isolated box (zero beyond the grid)
    int nslab;             // row slabs a sweep marches one after another (1: whole plane)
    int rows;              // rows per slab (n1 / nslab)
    double* b2;            // per system |b|^2 (mixed: written; FP64 continuation: read), or null
    int x_accum;           // FP64 continuation: x accumulates onto its current value and the
                           // tolerance is relative to b2[sys] instead of the start residual
};

// Element access through a uniform base pointer and a 32-bit unsigned offset, so loads and
// stores use the SGPR-base + 32-bit VGPR-offset addressing form (system size < 2^26 points).
template <typename V>
__device__ __forceinline__ V ld(const V* base, unsigned idx) {
    return *reinterpret_cast<const V*>(reinterpret_cast<const char*>(base) + idx * unsigned(sizeof(V)));
}
template <typename V>
__device__ __forceinline__ void st(V* base, unsigned idx, V v) {
    *reinterpret_cast<V*>(reinterpret_cast<char*>(base) + idx * unsigned(sizeof(V))) = v;
}

#ifndef RPA_PREFETCH
#define RPA_PREFETCH 1
#endif

// Stencil distances whose LDS reads may be in flight together (4 reads each).
#ifndef RPA_STENCIL_GROUP
#define RPA_STENCIL_GROUP 1
#endif

__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// A workgroup-uniform double moved to scalar registers.  Reduction results are uniform by
// construction (every thread sums the same LDS entries in the same order), but the compiler
// cannot prove it for values read from LDS and would keep them in vector registers.
__device__ __forceinline__ double uniform(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane(int(b));
    const int hi = __builtin_amdgcn_readfirstlane(int(b >> 32));
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}

template <int NV>
__device__ __forceinline__ void wg_reduce(double (&v)[NV], double* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] += __shfl_xor(v[k], o, 64);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) red[wave * NV + k] = v[k];
    }
    lds_barrier();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += red[w * NV + k];
        v[k] = uniform(s);
    }
    lds_barrier();
}

// The columns (x, y) a thread owns in the current slab: thread t owns local columns
// t, t + BS, ... of the slab's rows [y0, y0 + rows); col is the global column y n0 + x, cyl the
// row inside the slab.
template <int C>
struct Cols {
    int col[C], cx[C], cyl[C];
    bool valid[C];
    int y0;
};

template <int C>
__device__ __forceinline__ void make_cols(const Args& a, int slab, int tid, int BS, Cols<C>& cl) {
    const int ps = a.rows * a.n0;
    cl.y0 = slab * a.rows;
#pragma unroll
    for (int i = 0; i < C; ++i) {
        const int t = tid + i * BS;
        cl.valid[i] = t < ps;
        const int tt = cl.valid[i] ? t : 0;
        cl.cx[i] = tt % a.n0;
        cl.cyl[i] = tt / a.n0;
        cl.col[i] = (cl.y0 + cl.cyl[i]) * a.n0 + cl.cx[i];
    }
}

// LDS plane layout: rows + 12 rows of RS >= n0 + 12 entries (RS a multiple of 8, so that a
// wave's reads stay free of bank conflicts where it crosses a row end).  Row r + 6 holds
// x = -6 .. n0+5 of slab row r, for r = -6 .. rows+5: the 6 ghost columns on each side hold
// the periodic images along x, the 6 rows above and below the slab hold the neighbouring
// rows (periodic images of the slab's own rows when the slab is the whole plane, rows of the
// other slabs loaded from memory otherwise), so every neighbour of a point is a fixed offset
// from it (+-k along x, +-k RS along y) and no wrap is computed in the stencil.  Rows outside
// the slab carry only the real columns (the stencil has no diagonal terms).
__device__ __forceinline__ int lds_center(int rs, int cx, int cyl) { return (cyl + 6) * rs + cx + 6; }

// Isolated box: ghost entries that lie beyond the walls stay at the zeros written at kernel
// start.  y ghosts are written here only when the slab is the whole plane.
template <typename Q2>
__device__ __forceinline__ void stage_point(Q2* L, int rs, int n0, int n1, int cx, int cyl, Q2 v,
                                            bool periodic, bool yghost) {
    const int c0 = lds_center(rs, cx, cyl);
    L[c0] = v;
    if (!periodic) return;
    if (cx < 6) L[c0 + n0] = v;
    if (cx >= n0 - 6) L[c0 - n0] = v;
    if (!yghost) return;
    if (cyl < 6) L[c0 + n1 * rs] = v;
    if (cyl >= n1 - 6) L[c0 - n1 * rs] = v;
}

// q = (A c) for one column: A = -1/2 Lap_h + V - eps - i omega; x/y neighbours from the
// LDS plane L, z neighbours from the queue entries Q[zc-6 .. zc+6][i].  The three axes share
// the weights, so each distance k costs one multiply-add per component.  Each k's four LDS
// reads are consumed before the next k's are issued (the empty asm ties the accumulators),
// which bounds the registers held by reads in flight.
template <typename R, typename Q2, int NQ, int C>
__device__ __forceinline__ typename Cplx<R>::type stencil(const Args& a, const Q2* __restrict__ L,
                                                          const Q2 (&Q)[NQ][C], int zc, int i,
                                                          int cx, int cy, R diag, R om) {
    const int RS = a.rs;
    const Q2* Lc = L + lds_center(RS, cx, cy);
    R ax = 0, ay = 0;
#pragma unroll
    for (int k = 1; k <= 6; ++k) {
        const Q2 a1 = Lc[k], a2 = Lc[-k];
        const Q2 b1 = Lc[k * RS], b2 = Lc[-k * RS];
        const Q2 c1 = Q[zc + k][i], c2 = Q[zc - k][i];
        ax += R(a.cw[k]) * (((R(a1.x) + R(a2.x)) + (R(b1.x) + R(b2.x))) + (R(c1.x) + R(c2.x)));
        ay += R(a.cw[k]) * (((R(a1.y) + R(a2.y)) + (R(b1.y) + R(b2.y))) + (R(c1.y) + R(c2.y)));
        if (k % RPA_STENCIL_GROUP == 0) asm volatile("" : "+v"(ax), "+v"(ay) :: "memory");
    }
    const Q2 c = Q[zc][i];
    return typename Cplx<R>::type{ax + diag * R(c.x) + om * R(c.y), ay + diag * R(c.y) - om * R(c.x)};
}

// Generic z-march over the thread's columns of one slab: lead.load(z, i, first) fetches
// what the queue entry of plane z needs (first: the plane's centre step has not run yet in
// this sweep), lead.make(buf) turns it into the queue value; cent.load(z, i) fetches what the
// centre step needs, cent.finish(buf, z, i, c, q) consumes the stencil result.  Loads for step
// s+1 are issued before step s computes.  With SLAB, the 6 rows above and below the slab are
// loaded for every centre plane (lead.load_at at a global column) and staged next to the
// slab's own rows.
// Q is the caller's queue.  With warm = true it already holds planes -6 .. 5 (mod n2) of the
// lead vector in Q[0..11] and the warm-up is skipped.  On return Q[0..11] holds planes
// -6 .. 5 of the lead vector again (the queue has wrapped around the periodic z axis).
template <typename R, typename Q2, int C, int Z, bool SLAB, class Lead, class Cent>
__device__ __forceinline__ void march(const Args& a, const Cols<C>& cl, Q2* lds, double eps_n,
                                      Lead& lead, Cent& cent, Q2 (&Q)[12 + Z][C], bool warm) {
    constexpr int NQ = 12 + Z;
    const int n2 = a.n2, P = a.P;
    const R om = R(a.omega);
    const int tid = threadIdx.x;
    // slab mode: thread t < 12 n0 loads halo entry t of each centre plane (the launch has
    // at least 12 n0 threads): rows y0-6 .. y0-1 for t < 6 n0, rows y0+rows .. y0+rows+5 after
    const int nh = SLAB ? 12 * a.n0 : 0;
    const bool hv = tid < nh;
    int hx = 0, lr = 0;
    unsigned hcol = 0;
    bool hin = false, hdone = false;
    if (SLAB && hv) {
        const int hr = tid / a.n0;
        hx = tid - hr * a.n0;
        lr = (hr < 6) ? hr - 6 : a.rows + hr - 6;
        int gy = cl.y0 + lr;
        if (a.periodic) {
            gy += (gy < 0) ? a.n1 : 0;
            gy -= (gy >= a.n1) ? a.n1 : 0;
            hin = true;
        } else {
            hin = gy >= 0 && gy < a.n1;      // isolated box: rows beyond the walls are zero
        }
        hcol = unsigned(gy * a.n0 + hx);
        // slabs run in order within a sweep: a row below the slab's first row belongs to a
        // slab already marched in this sweep (lead.load_done may read what that slab wrote)
        hdone = hin && gy < cl.y0;
    }
    typename Lead::Buf LB[Z][C];
    typename Cent::Buf CB[Z][C];
    typename Lead::Buf HB[Z];
    auto halo_load = [&](int zc) -> typename Lead::Buf {
        if (!hin) return typename Lead::Buf{};
        return hdone ? lead.load_done(zc, hcol) : lead.load_at(zc, hcol);
    };
    // warm-up: push planes -6 .. 5 through the top of the queue, Z at a time
#pragma unroll 1
    for (int w = 0; w < (warm ? 0 : 12 / Z); ++w) {
#pragma unroll
        for (int zz = 0; zz < Z; ++zz) {
            const int zu = w * Z + zz - 6;
            const int z = zu + ((zu < 0) ? n2 : 0);
            const bool in = a.periodic || zu >= 0;      // box: planes below 0 are zero
#pragma unroll
            for (int i = 0; i < C; ++i)
                Q[12 + zz][i] = (cl.valid[i] && in) ? lead.make(lead.load(z, i, true)) : Q2{0, 0};
        }
#pragma unroll
        for (int s = 0; s < 12; ++s)
#pragma unroll
            for (int i = 0; i < C; ++i) Q[s][i] = Q[s + Z][i];
    }
#pragma unroll
    for (int zz = 0; zz < Z; ++zz) {
        int z = 6 + zz;
        z -= (z >= n2) ? n2 : 0;
#pragma unroll
        for (int i = 0; i < C; ++i) {
            if (cl.valid[i]) {
                LB[zz][i] = lead.load(z, i, true);
                CB[zz][i] = cent.load(zz, i);
            }
        }
        if (SLAB) HB[zz] = halo_load(zz);
    }
    const int nsteps = n2 / Z;
#pragma unroll 1
    for (int st = 0; st < nsteps; ++st) {
        const int zo = st * Z;
        typename Cent::Buf CC[Z][C];
        Q2 HC[Z];
        if (!RPA_PREFETCH && st > 0) {
#pragma unroll
            for (int zz = 0; zz < Z; ++zz) {
                const int zu = zo + 6 + zz;
                const int z = zu - ((zu >= n2) ? n2 : 0);
                const bool in = a.periodic || zu < n2;      // box: planes beyond n2-1 are zero
#pragma unroll
                for (int i = 0; i < C; ++i)
                    if (cl.valid[i]) {
                        LB[zz][i] = in ? lead.load(z, i, zu < n2 || zu - n2 >= zo)
                                       : typename Lead::Buf{};
                        CB[zz][i] = cent.load(zo + zz, i);
                    }
                if (SLAB) HB[zz] = halo_load(zo + zz);
            }
        }
#pragma unroll
        for (int zz = 0; zz < Z; ++zz) {
#pragma unroll
            for (int i = 0; i < C; ++i) {
                Q[12 + zz][i] = cl.valid[i] ? lead.make(LB[zz][i]) : Q2{0, 0};
                CC[zz][i] = CB[zz][i];
            }
            if (SLAB) HC[zz] = lead.make(HB[zz]);
        }
        if (RPA_PREFETCH && st + 1 < nsteps) {
#pragma unroll
            for (int zz = 0; zz < Z; ++zz) {
                const int zu = zo + Z + 6 + zz;          // < 2 n2 since n2 >= 12, Z <= 4
                const int z = zu - ((zu >= n2) ? n2 : 0);
                const bool in = a.periodic || zu < n2;
#pragma unroll
                for (int i = 0; i < C; ++i) {
                    if (cl.valid[i]) {
                        // planes below zo have had their centre step; this step's
                        // centres run after these loads are issued
                        LB[zz][i] = in ? lead.load(z, i, zu < n2 || zu - n2 >= zo)
                                       : typename Lead::Buf{};
                        CB[zz][i] = cent.load(zo + Z + zz, i);
                    }
                }
                if (SLAB) HB[zz] = halo_load(zo + Z + zz);
            }
        }
        const int PL = (a.rows + 12) * a.rs;     // slab plane with ghost rows and columns
        Q2* L = lds + (a.nbuf == 2 ? (st & 1) : 0) * Z * PL;
#pragma unroll
        for (int zz = 0; zz < Z; ++zz) {
#pragma unroll
            for (int i = 0; i < C; ++i)
                if (cl.valid[i])
                    stage_point(L + zz * PL, a.rs, a.n0, a.n1, cl.cx[i], cl.cyl[i], Q[6 + zz][i],
                                a.periodic != 0, !SLAB);
            // halo rows, with their x ghosts when periodic
            if (SLAB && hv)
                stage_point(L + zz * PL, a.rs, a.n0, a.n1, hx, lr, HC[zz], a.periodic != 0, false);
        }
        lds_barrier();
#pragma unroll
        for (int zz = 0; zz < Z; ++zz) {
#pragma unroll
            for (int i = 0; i < C; ++i) {
                if (!cl.valid[i]) continue;
                const unsigned idx = unsigned((zo + zz) * P + cl.col[i]);
                // float32 sweeps read the float32 copy of V_loc (the mixed driver always passes
                // it); the diagonal is a float32 value either way
                R diag;
                if constexpr (std::is_same<R, float>::value)
                    diag = R(a.cw[0] - eps_n) + ld(a.vloc32, idx);
                else
                    diag = R(a.cw[0] + ld(a.vloc, idx) - eps_n);
                const auto q = stencil<R, Q2, NQ, C>(a, L + zz * PL, Q, 6 + zz, i, cl.cx[i],
                                                     cl.cyl[i], diag, om);
                cent.finish(CC[zz][i], zo + zz, i, Q[6 + zz][i], q);
                // one column at a time: keeps the next column's LDS reads (and registers)
                // behind this column's stores
                if (C > 1) asm volatile("" ::: "memory");
            }
        }
        if (a.nbuf == 1) lds_barrier();      // single buffer: reads done before the next write
#pragma unroll
        for (int s = 0; s < 12; ++s)
#pragma unroll
            for (int i = 0; i < C; ++i) Q[s][i] = Q[s + Z][i];
    }
}

struct Empty {};

// ---------------------------------------------------------------- sweep 1 (sigma)
template <typename T2, int C, typename RA, bool PN>
struct LeadPnew {
    struct Buf { T2 r, p; };
    const T2* r; const T2* pa; const T2* pn; int P; const int* col; bool first; double dbr, dbi;
    __device__ Buf load(int z, int i, bool) const { return load_at(z, unsigned(col[i])); }
    __device__ Buf load_at(int z, unsigned gcol) const {
        const unsigned idx = unsigned(z * P) + gcol;
        Buf b;
        b.r = ld(r, idx);
        b.p = first ? T2{0, 0} : ld(pa, idx);
        return b;
    }
    // a row of a slab marched earlier in this sweep: with PN its p_new is read from pn (the
    // value make() would compute, rounded the same way), one load instead of two; make()
    // returns it unchanged since p = 0
    __device__ Buf load_done(int z, unsigned gcol) const {
        if constexpr (PN) {
            Buf b;
            b.r = ld(pn, unsigned(z * P) + gcol);
            b.p = T2{0, 0};
            return b;
        } else {
            return load_at(z, gcol);
        }
    }
    // p_new = r + beta p in the arithmetic precision, rounded once to the state precision
    __device__ T2 make(const Buf& b) const {
        using S = decltype(T2{}.x);
        const RA br_ = RA(dbr), bi_ = RA(dbi);
        return T2{S(RA(b.r.x) + br_ * RA(b.p.x) - bi_ * RA(b.p.y)),
                  S(RA(b.r.y) + br_ * RA(b.p.y) + bi_ * RA(b.p.x))};
    }
};
template <typename T2, int C>
struct CentSigma {
    using Buf = Empty;
    T2* pb; int P; const int* col; bool first;
    double acc[7];   // sigma re/im, |p|^2, |q|^2, rho0 re/im, |r0|^2
    __device__ Buf load(int, int) const { return Buf{}; }
    template <typename Q>
    __device__ void finish(const Buf&, int z, int i, T2 c, Q q) {
        acc[0] += double(c.x) * q.x - double(c.y) * q.y;
        acc[1] += double(c.x) * q.y + double(c.y) * q.x;
        acc[2] += double(c.x) * c.x + double(c.y) * c.y;
        acc[3] += double(q.x) * q.x + double(q.y) * q.y;
        if (first) {
            acc[4] += double(c.x) * c.x - double(c.y) * c.y;
            acc[5] += 2.0 * double(c.x) * c.y;
            acc[6] += double(c.x) * c.x + double(c.y) * c.y;
        }
        st(pb, unsigned(z * P + col[i]), c);
    }
};

// ---------------------------------------------------------------- sweep 2 (update)
template <typename T2>
struct LeadLoad {
    using Buf = T2;
    const T2* v; int P; const int* col;
    __device__ Buf load(int z, int i, bool) const { return ld(v, unsigned(z * P + col[i])); }
    __device__ Buf load_at(int z, unsigned gcol) const { return ld(v, unsigned(z * P) + gcol); }
    __device__ Buf load_done(int z, unsigned gcol) const { return load_at(z, gcol); }
    __device__ T2 make(const Buf& b) const { return b; }
};
// x stored as XS (double: real part only, double2: complex FP64, float2: complex64 x_lo);
// the updates run in the arithmetic precision RA and round once when stored
template <typename T2, typename XS, typename RA>
struct CentUpdate {
    struct Buf { T2 r; XS x; };
    T2* r; XS* x; int P; const int* col; bool xzero; double ar, ai;
    double acc[3];   // rho' re/im, |r|^2
    __device__ Buf load(int z, int i) const {
        const unsigned idx = unsigned(z * P + col[i]);
        Buf b;
        b.r = ld(r, idx);
        if (xzero) b.x = XS{}; else b.x = ld(x, idx);
        return b;
    }
    template <typename Q>
    __device__ void finish(const Buf& bf, int z, int i, T2 c, Q q) {
        using S = decltype(T2{}.x);
        const unsigned idx = unsigned(z * P + col[i]);
        const RA a_r = RA(ar), a_i = RA(ai);
        T2 rv;
        rv.x = S(RA(bf.r.x) - (a_r * RA(q.x) - a_i * RA(q.y)));
        rv.y = S(RA(bf.r.y) - (a_r * RA(q.y) + a_i * RA(q.x)));
        st(r, idx, rv);
        XS xv = bf.x;
        if constexpr (std::is_same<XS, double>::value) {
            xv += double(a_r) * c.x - double(a_i) * c.y;
        } else {
            using XE = decltype(XS{}.x);
            xv.x = XE(RA(xv.x) + (a_r * RA(c.x) - a_i * RA(c.y)));
            xv.y = XE(RA(xv.y) + (a_r * RA(c.y) + a_i * RA(c.x)));
        }
        st(x, idx, xv);
        acc[0] += double(rv.x) * rv.x - double(rv.y) * rv.y;
        acc[1] += 2.0 * double(rv.x) * rv.y;
        acc[2] += double(rv.x) * rv.x + double(rv.y) * rv.y;
    }
};

// ---------------------------------------------------------------- reliable update (mixed)
// One z-march over x_lo with a complex64 queue; the stencil promotes every value to float64.
// The centre step adds x_lo to x_hi, subtracts A x_lo from r_hi, stores both and
// r = complex64(r_hi), and accumulates r^T r (of the stored complex64 r) and |r_hi|^2.
// Every address is read and written by its own thread only.
struct LeadXlo {
    using Buf = float2;
    const float2* xlo; int P; const int* col;
    __device__ Buf load(int z, int i, bool) const { return ld(xlo, unsigned(z * P + col[i])); }
    __device__ Buf load_at(int z, unsigned gcol) const { return ld(xlo, unsigned(z * P) + gcol); }
    __device__ Buf load_done(int z, unsigned gcol) const { return load_at(z, gcol); }
    __device__ float2 make(const Buf& b) const { return b; }
};
struct CentRhi {
    struct Buf { double2 rh, xh; };
    double2* rhi; double2* xhi; float2* r; int P; const int* col; bool xhi_zero;
    double acc[3];   // rho re/im, |r_hi|^2
    __device__ Buf load(int z, int i) const {
        const unsigned idx = unsigned(z * P + col[i]);
        Buf b;
        b.rh = ld(rhi, idx);
        b.xh = xhi_zero ? double2{0.0, 0.0} : ld(xhi, idx);
        return b;
    }
    __device__ void finish(const Buf& bf, int z, int i, float2 c, double2 q) {
        const unsigned idx = unsigned(z * P + col[i]);
        const double2 rh{bf.rh.x - q.x, bf.rh.y - q.y};
        st(rhi, idx, rh);
        st(xhi, idx, double2{bf.xh.x + double(c.x), bf.xh.y + double(c.y)});
        const float2 rv{float(rh.x), float(rh.y)};
        st(r, idx, rv);
        acc[0] += double(rv.x) * rv.x - double(rv.y) * rv.y;
        acc[1] += 2.0 * double(rv.x) * rv.y;
        acc[2] += rh.x * rh.x + rh.y * rh.y;
    }
};

// x_hi <- x_hi + x_lo over the thread's own columns (a solve that stops without a final
// reliable update: a zero right-hand side, whose x_hi is written only here)
template <int C>
__device__ __forceinline__ void fold_xlo(const Args& a, const int (&col)[C], const bool (&valid)[C],
                                         double2* xhi, const float2* xlo, bool xhi_zero) {
    for (int z = 0; z < a.n2; ++z) {
#pragma unroll
        for (int i = 0; i < C; ++i) {
            if (!valid[i]) continue;
            const unsigned idx = unsigned(z * a.P + col[i]);
            const float2 l = ld(xlo, idx);
            double2 h = xhi_zero ? double2{0.0, 0.0} : ld(xhi, idx);
            h.x += double(l.x);
            h.y += double(l.y);
            st(xhi, idx, h);
        }
    }
}

// ---------------------------------------------------------------- the solver
// T: state precision (double: FP64 path, float: mixed); XS: type of the stored solution in
// the FP64 path (double = real part only, double2 = complex); ignored when T = float.
// OCC = minimum resident waves per SIMD the register allocation must allow (0: derived from
// BSMAX alone); higher values cap the registers so that two workgroups share a CU.
// SLAB: the plane is marched in a.nslab row slabs one after another (large planes whose
// whole-plane columns would not fit in registers); otherwise a.nslab = 1 and a.rows = n1.
template <typename T, typename XS, int C, int Z, int BSMAX, int OCC = 0, bool SLAB = false>
__global__ __attribute__((amdgpu_flat_work_group_size(64, BSMAX),
                          amdgpu_waves_per_eu(OCC > 0 ? OCC : 1, 8)))
void cocg_wg(Args a_in) {
    using T2 = typename Cplx<T>::type;
    using RA = typename Arith<T>::type;
    constexpr bool MIXED = std::is_same<T, float>::value;
    // sweep 1 of the FP64 slab kernel reads the halo rows of slabs already marched from their
    // p_new (measured at 48^3: 3.4% faster; the complex64 kernel, which saves half the bytes
    // per row, ran 4.8% slower with the extra memory barrier per slab and keeps r and p)
    constexpr bool PN = !MIXED;
    // Dispatch order: the host passes a permutation that starts the systems expected to need
    // the most iterations first (longest-first list scheduling: the easy ones then fill the
    // CUs behind them instead of leaving a long single-system tail).  Without one, orbitals
    // closest to the gap (largest n, smallest shifted gap) go first: system s = n + ns*j,
    // workgroup b takes n = ns-1 - b / nvec, j = b % nvec.
    const int nvec_l = int(gridDim.x) / a_in.ns;
    const int bid = blockIdx.x;
    const int sys = a_in.order ? a_in.order[bid]
                  : (nvec_l > 0 && int(gridDim.x) % a_in.ns == 0)
                        ? (a_in.ns - 1 - bid / nvec_l) + a_in.ns * (bid % nvec_l)
                        : bid;
    Args a = a_in;
    if (a_in.omega_v) a.omega = a_in.omega_v[sys / a_in.ns];
    const int tid = threadIdx.x, BS = blockDim.x;
    const int n0 = a.n0, P = a.P;
    const int64_t off = int64_t(sys) * a.nd;
    T2* r = reinterpret_cast<T2*>(a.r) + off;
    T2* pa = reinterpret_cast<T2*>(a.pa) + off;
    T2* pb = reinterpret_cast<T2*>(a.pb) + off;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* red = reinterpret_cast<double*>(smem_raw);                // 16 waves x 8
    unsigned char* planes = smem_raw + 16 * 8 * sizeof(double);
    const double eps_n = a.eps[sys % a.ns];

    const int nslab = SLAB ? a.nslab : 1;
    Cols<C> cl;
    make_cols<C>(a, 0, tid, BS, cl);
    // In slab mode a sweep reads rows of the swept vector that other threads wrote in the
    // previous sweep: the end of every sweep is a workgroup-wide memory barrier.
    auto slab_sync = [&]() {
        if (SLAB) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_s_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        }
    };
    // next slab: new columns; the previous slab's last LDS reads finish before the first write
    auto next_slab = [&](int sl) {
        if (SLAB) {
            make_cols<C>(a, sl, tid, BS, cl);
            if (sl > 0) lds_barrier();
        }
    };
    // the same for sweep 1, whose halo rows of earlier slabs are read from the p_new those
    // slabs wrote: their global stores are made visible to the whole workgroup as well
    auto next_slab_pn = [&](int sl) {
        if (SLAB) {
            make_cols<C>(a, sl, tid, BS, cl);
            if (sl > 0) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                __builtin_amdgcn_s_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            }
        }
    };

    if (!a.periodic) {
        // isolated box: every ghost entry of the staged planes reads zero; stage_point never
        // writes x ghosts in this mode and writes the y ghosts only as zero halo rows, so
        // clearing the plane buffers once suffices
        const int nent = a.nbuf * Z * (a.rows + 12) * a.rs;
        double2* pl = reinterpret_cast<double2*>(planes);
        for (int e = tid; e < nent; e += BS) pl[e] = double2{0.0, 0.0};
        lds_barrier();
    }

    double rho_re = 0, rho_im = 0, bb = 0, beta_re = 0, beta_im = 0, rr_ref = 0, tgt2 = 0;
    int it = 0, st = 0, nref = 0, it_ref = 0;
    bool xlo_zero = true, xhi_zero = true, done = false;
    bool cold = false;     // the queue was dropped (reliable update): sweep 1 reloads it
    // Queue of the swept vector, carried from sweep to sweep: after sweep 1 it holds planes
    // -6 .. 5 of the new p, which is what sweep 2 starts from; after sweep 2 it still holds
    // those planes of p, and the next sweep 1 starts from r' + beta' p on them.
    T2 Q[12 + Z][C];

    while (!done) {
        const bool first = (it == 0);
        // ---------------------------------------------------------- sweep 1
        // (isolated box: the queue left by a sweep holds the planes past the top wall, not the
        // planes below the bottom one, so every sweep starts cold)
        const bool carry = !SLAB && !first && !cold && a.periodic;
        if (carry) {
            // warm start of sweep 1 from the queue: p_new = r + beta p on planes -6 .. 5,
            // four planes at a time
            const RA br = RA(beta_re), bi = RA(beta_im);
#pragma unroll
            for (int s0 = 0; s0 < 12; s0 += 4) {
                T2 rw[4][C];
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    int z = s0 + s - 6;
                    z += (z < 0) ? a.n2 : 0;
#pragma unroll
                    for (int i = 0; i < C; ++i)
                        rw[s][i] = cl.valid[i] ? ld(r, unsigned(z * P + cl.col[i])) : T2{0, 0};
                }
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int i = 0; i < C; ++i) {
                        const T2 pv = Q[s0 + s][i];
                        Q[s0 + s][i] = T2{T(RA(rw[s][i].x) + br * RA(pv.x) - bi * RA(pv.y)),
                                          T(RA(rw[s][i].y) + br * RA(pv.y) + bi * RA(pv.x))};
                    }
            }
        }
        LeadPnew<T2, C, RA, PN> l1{r, pa, pb, P, cl.col, first, beta_re, beta_im};
        CentSigma<T2, C> c1{pb, P, cl.col, first, {0, 0, 0, 0, 0, 0, 0}};
        for (int sl = 0; sl < nslab; ++sl) {
            if constexpr (PN)
                next_slab_pn(sl);
            else
                next_slab(sl);
            march<RA, T2, C, Z, SLAB>(a, cl, reinterpret_cast<T2*>(planes), eps_n, l1, c1, Q,
                                      carry);
        }
        slab_sync();
        cold = false;
        wg_reduce<7>(c1.acc, red);
        if (first) {
            rho_re = c1.acc[4];
            rho_im = c1.acc[5];
            bb = c1.acc[6];
            rr_ref = bb;
            // stopping target |r|^2 <= tol^2 |b|^2; a continuation starts from the residual of
            // an earlier solve, so its reference is that solve's |b|^2
            tgt2 = uniform(a.tol2 * ((a.x_accum && a.b2) ? a.b2[sys] : bb));
        }
        const bool zero_rhs = first && !(bb > 0.0);
        bool breakdown = false;
        double alpha_re = 0, alpha_im = 0;
        if (!zero_rhs) {
            ++it;
            const double s2 = c1.acc[0] * c1.acc[0] + c1.acc[1] * c1.acc[1];
            if (!(s2 > a.bd_tol * a.bd_tol * c1.acc[2] * c1.acc[3])) {
                breakdown = true;
            } else {
                alpha_re = uniform((rho_re * c1.acc[0] + rho_im * c1.acc[1]) / s2);
                alpha_im = uniform((rho_im * c1.acc[0] - rho_re * c1.acc[1]) / s2);
            }
        }
        // ---------------------------------------------------------- sweep 2
        double acc2[3];
        {
            LeadLoad<T2> l2{pb, P, cl.col};
            if constexpr (MIXED) {
                CentUpdate<T2, float2, RA> c2{r, reinterpret_cast<float2*>(a.xlo) + off, P, cl.col,
                                          xlo_zero, alpha_re, alpha_im, {0, 0, 0}};
                for (int sl = 0; sl < nslab; ++sl) {
                    next_slab(sl);
                    march<RA, T2, C, Z, SLAB>(a, cl, reinterpret_cast<T2*>(planes), eps_n, l2, c2,
                                              Q, !SLAB && a.periodic != 0);
                }
                slab_sync();
                wg_reduce<3>(c2.acc, red);
                acc2[0] = c2.acc[0]; acc2[1] = c2.acc[1]; acc2[2] = c2.acc[2];
            } else {
                CentUpdate<T2, XS, RA> c2{r, reinterpret_cast<XS*>(a.x) + off, P, cl.col,
                                      first && !a.x_accum, alpha_re, alpha_im, {0, 0, 0}};
                for (int sl = 0; sl < nslab; ++sl) {
                    next_slab(sl);
                    march<RA, T2, C, Z, SLAB>(a, cl, reinterpret_cast<T2*>(planes), eps_n, l2, c2,
                                              Q, !SLAB && a.periodic != 0);
                }
                slab_sync();
                wg_reduce<3>(c2.acc, red);
                acc2[0] = c2.acc[0]; acc2[1] = c2.acc[1]; acc2[2] = c2.acc[2];
            }
        }
        xlo_zero = false;
        // mixed: reliable update (group-wise residual replacement): x_hi += x_lo and
        // r_hi -= A x_lo in float64, then r = complex64(r_hi)
        auto reliable_update = [&]() {
            // drop the carried queue so that its registers are free for this sweep; the next
            // sweep 1 reloads its first planes from memory
#pragma unroll
            for (int q = 0; q < 12 + Z; ++q)
#pragma unroll
                for (int i = 0; i < C; ++i) Q[q][i] = T2{0, 0};
            cold = true;
            float2 Qx[12 + 1][C];
            LeadXlo lx{reinterpret_cast<const float2*>(a.xlo) + off, P, cl.col};
            CentRhi cr{reinterpret_cast<double2*>(a.rhi) + off,
                       reinterpret_cast<double2*>(a.x) + off, reinterpret_cast<float2*>(r),
                       P, cl.col, xhi_zero, {0, 0, 0}};
            for (int sl = 0; sl < nslab; ++sl) {
                next_slab(sl);
                march<double, float2, C, 1, SLAB>(a, cl, reinterpret_cast<float2*>(planes),
                                                  eps_n, lx, cr, Qx, false);
            }
            slab_sync();
            wg_reduce<3>(cr.acc, red);
            xhi_zero = false;
            xlo_zero = true;
            ++nref;
            acc2[0] = cr.acc[0]; acc2[1] = cr.acc[1]; acc2[2] = cr.acc[2];
            rr_ref = acc2[2];
            it_ref = it;
        };
        if (zero_rhs) {
            done = true;
        } else if (breakdown) {
            // mixed: a final reliable update leaves x_hi and the exact r_hi = b - A x_hi, from
            // which the host restarts the system in FP64 (as after the iteration cap)
            if constexpr (MIXED) reliable_update();
            st = 2;
            done = true;
        } else {
            bool conv = false;
            bool updated = false;
            if constexpr (MIXED) {
                // reliable update when the complex64 residual fell by refine_tol or hit tol,
                // and at the iteration cap (so that a stopped solve leaves x_hi and the exact
                // r_hi = b - A x_hi for an FP64 continuation)
                if (acc2[2] <= tgt2 || it >= a.max_iter ||
                    (acc2[2] <= a.refine2 * rr_ref && it - it_ref >= a.refine_gap)) {
                    reliable_update();
                    updated = true;
                    conv = acc2[2] <= tgt2;
                }
            } else {
                conv = acc2[2] <= tgt2;
            }
            if (conv) {
                done = true;
            } else if (it >= a.max_iter) {
                st = 1;
                done = true;
            } else {
                const double n2r = acc2[0] * acc2[0] + acc2[1] * acc2[1];
                if (!(n2r > a.bd_tol * a.bd_tol * acc2[2] * acc2[2])) {
                    if constexpr (MIXED) {
                        if (!updated) reliable_update();
                    }
                    st = 2;
                    done = true;
                } else {
                    const double rr = rho_re * rho_re + rho_im * rho_im;
                    beta_re = uniform((acc2[0] * rho_re + acc2[1] * rho_im) / rr);
                    beta_im = uniform((acc2[1] * rho_re - acc2[0] * rho_im) / rr);
                    rho_re = acc2[0];
                    rho_im = acc2[1];
                    T2* t = pa;
                    pa = pb;
                    pb = t;
                }
            }
        }
    }
    if constexpr (MIXED) {
        // the solution lives in x_hi: fold the last partial solution if it is pending
        if (!xlo_zero) {
            for (int sl = 0; sl < nslab; ++sl) {
                if (SLAB) make_cols<C>(a, sl, tid, BS, cl);
                fold_xlo<C>(a, cl.col, cl.valid, reinterpret_cast<double2*>(a.x) + off,
                            reinterpret_cast<const float2*>(a.xlo) + off, xhi_zero);
            }
        }
    }
    if (tid == 0) {
        a.iters[sys] = it;
        a.status[sys] = st;
        if (a.refinements) a.refinements[sys] = nref;
        if (MIXED && a.b2) a.b2[sys] = bb;
    }
}

}  // namespace cocg
}  // namespace rpa
