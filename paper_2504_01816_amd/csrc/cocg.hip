// Batched COCG for the shifted Sternheimer systems (H - eps_n - i omega) x = b
// (Sec. 3: COCG, the CG variant with the unconjugated bilinear form; Eq. 9).
//
// Design (gfx950):
//  * One workgroup owns one system for its whole solve.  The two reductions of each COCG
//    iteration (sigma = p^T A p, then rho = r^T r) are workgroup-local, so a system runs
//    all its iterations inside one launch with no host round trip and no grid-wide
//    barrier.  Systems converge independently; a finished workgroup frees its CU slot and
//    the hardware dispatcher starts the next system, which is the active-set compaction.
//  * Each iteration is two streaming sweeps over the system:
//      sweep 1: p <- r + beta p (written to the other p buffer), q = A p, reduce
//               sigma = p^T q, |p|^2, |q|^2;
//      sweep 2: q = A p recomputed (no q array is stored), x <- x + alpha p,
//               r <- r - alpha q, reduce rho' = r^T r and |r|^2.
//    Traffic per point per iteration (complex128, x kept real): 48 + 64 B.
//  * A sweep marches along z.  Thread t owns columns t, t+BS, ... of the x-y plane and
//    keeps the 13 planes z-6..z+6 of p for its columns in registers; the current plane is
//    staged in LDS (two buffers, one barrier per plane) for the x and y neighbours.
//    Loads and stores are coalesced along x.
//  * Reductions are fixed-order (wave butterfly, then waves in order): results are
//    bitwise reproducible run to run.
//
// Layout: state arrays are system-major, nsys x N_d, complex interleaved (re, im).
// Grid constraints: n2 >= 12 (the marching queue), n0, n1 >= 7 (single periodic wrap).
#include "internal.h"

namespace rpa {
namespace {

template <typename T> struct Cplx;
template <> struct Cplx<double> { using type = double2; };
template <> struct Cplx<float> { using type = float2; };

struct CocgArgs {
    int n0, n1, n2, P;
    double cw[7];          // cw[k] = -1/2 w_k / h^2 for k >= 1; cw[0] = -1/2 * 3 w_0 / h^2
    const double* vloc;
    const double* eps;
    int ns;
    double omega;
    double tol2;
    int max_iter;
    double bd_tol;
    int64_t nd;
    void* r;
    void* pa;
    void* pb;
    void* x;
    int* iters;
    int* status;
};

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
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += red[w * NV + k];
        v[k] = s;
    }
    __syncthreads();
}

template <typename T2>
__device__ __forceinline__ T2 cmul(T2 a, T2 b) {
    return T2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// q = A c for one column: A = -1/2 Lap_h + V - eps - i omega, with the x/y neighbours in
// the LDS plane L and the z neighbours in the register queue Q[0..12][i].
template <typename T, typename T2, int C>
__device__ __forceinline__ T2 apply_a(const CocgArgs& a, const T2* __restrict__ L,
                                      const T2 (&Q)[13][C], int i, int cx, int cy, T diag,
                                      T om) {
    const int n0 = a.n0, n1 = a.n1;
    T ax = 0, ay = 0;
#pragma unroll
    for (int k = 1; k <= 6; ++k) {
        int xp = cx + k; xp -= (xp >= n0) ? n0 : 0;
        int xm = cx - k; xm += (xm < 0) ? n0 : 0;
        int yp = cy + k; yp -= (yp >= n1) ? n1 : 0;
        int ym = cy - k; ym += (ym < 0) ? n1 : 0;
        const T2 a1 = L[cy * n0 + xp], a2 = L[cy * n0 + xm];
        const T2 b1 = L[yp * n0 + cx], b2 = L[ym * n0 + cx];
        const T2 c1 = Q[6 + k][i], c2 = Q[6 - k][i];
        const T w = T(a.cw[k]);
        ax += w * ((a1.x + a2.x) + (b1.x + b2.x) + (c1.x + c2.x));
        ay += w * ((a1.y + a2.y) + (b1.y + b2.y) + (c1.y + c2.y));
    }
    const T2 c = Q[6][i];
    return T2{ax + diag * c.x + om * c.y, ay + diag * c.y - om * c.x};
}

template <typename T, int C, int BSMAX, bool XC>
__global__ __launch_bounds__(BSMAX) void cocg_wg(CocgArgs a) {
    using T2 = typename Cplx<T>::type;
    const int sys = blockIdx.x;
    const int tid = threadIdx.x, BS = blockDim.x;
    const int n0 = a.n0, n2 = a.n2, P = a.P;
    const int64_t off = int64_t(sys) * a.nd;
    T2* __restrict__ r = reinterpret_cast<T2*>(a.r) + off;
    T2* pa = reinterpret_cast<T2*>(a.pa) + off;
    T2* pb = reinterpret_cast<T2*>(a.pb) + off;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T2* lds = reinterpret_cast<T2*>(smem_raw);
    double* red = reinterpret_cast<double*>(smem_raw + 2 * size_t(P) * sizeof(T2));

    const double eps_n = a.eps[sys % a.ns];
    const T om = T(a.omega);

    int col[C], cx[C], cy[C];
    bool valid[C];
#pragma unroll
    for (int i = 0; i < C; ++i) {
        col[i] = tid + i * BS;
        valid[i] = col[i] < P;
        const int cc = valid[i] ? col[i] : 0;
        cx[i] = cc % n0;
        cy[i] = cc / n0;
    }

    T2 Q[13][C];
    double rho_re = 0, rho_im = 0, bb = 0;
    double beta_re = 0, beta_im = 0;
    int it = 0, st = 0;
    bool done = false;

    while (!done) {
        const bool first = (it == 0);
        // ------------------------------------------------------------ sweep 1
        auto load_pnew = [&](int z, int i) -> T2 {
            const int64_t idx = int64_t(z) * P + col[i];
            const T2 rv = r[idx];
            if (first) return rv;
            const T2 po = pa[idx];
            return T2{rv.x + T(beta_re) * po.x - T(beta_im) * po.y,
                      rv.y + T(beta_re) * po.y + T(beta_im) * po.x};
        };
        double acc1[7] = {0, 0, 0, 0, 0, 0, 0};  // sigma re/im, |p|^2, |q|^2, rho0 re/im, bb
#pragma unroll
        for (int s = 0; s < 12; ++s) {
            int z = s - 6;
            z += (z < 0) ? n2 : 0;
#pragma unroll
            for (int i = 0; i < C; ++i) Q[s][i] = valid[i] ? load_pnew(z, i) : T2{0, 0};
        }
        for (int zo = 0; zo < n2; ++zo) {
            int zl = zo + 6;
            zl -= (zl >= n2) ? n2 : 0;
#pragma unroll
            for (int i = 0; i < C; ++i) Q[12][i] = valid[i] ? load_pnew(zl, i) : T2{0, 0};
            T2* L = lds + (zo & 1) * P;
#pragma unroll
            for (int i = 0; i < C; ++i)
                if (valid[i]) L[col[i]] = Q[6][i];
            __syncthreads();
#pragma unroll
            for (int i = 0; i < C; ++i) {
                if (!valid[i]) continue;
                const int64_t idx = int64_t(zo) * P + col[i];
                const T diag = T(a.cw[0] + a.vloc[idx] - eps_n);
                const T2 q = apply_a<T, T2, C>(a, L, Q, i, cx[i], cy[i], diag, om);
                const T2 c = Q[6][i];
                acc1[0] += double(c.x) * q.x - double(c.y) * q.y;
                acc1[1] += double(c.x) * q.y + double(c.y) * q.x;
                acc1[2] += double(c.x) * c.x + double(c.y) * c.y;
                acc1[3] += double(q.x) * q.x + double(q.y) * q.y;
                if (first) {
                    acc1[4] += double(c.x) * c.x - double(c.y) * c.y;
                    acc1[5] += 2.0 * double(c.x) * c.y;
                    acc1[6] += double(c.x) * c.x + double(c.y) * c.y;
                }
                pb[idx] = c;
            }
#pragma unroll
            for (int s = 0; s < 12; ++s)
#pragma unroll
                for (int i = 0; i < C; ++i) Q[s][i] = Q[s + 1][i];
        }
        wg_reduce<7>(acc1, red);
        if (first) {
            rho_re = acc1[4];
            rho_im = acc1[5];
            bb = acc1[6];
        }
        double alpha_re = 0, alpha_im = 0;
        bool zero_rhs = first && !(bb > 0.0);
        bool breakdown = false;
        if (!zero_rhs) {
            ++it;
            const double s2 = acc1[0] * acc1[0] + acc1[1] * acc1[1];
            if (!(s2 > a.bd_tol * a.bd_tol * acc1[2] * acc1[3])) {
                breakdown = true;
            } else {
                // alpha = rho / sigma
                alpha_re = (rho_re * acc1[0] + rho_im * acc1[1]) / s2;
                alpha_im = (rho_im * acc1[0] - rho_re * acc1[1]) / s2;
            }
        }
        // ------------------------------------------------------------ sweep 2
        const T ar = T(alpha_re), ai = T(alpha_im);
        double acc2[3] = {0, 0, 0};  // rho' re/im, |r|^2
#pragma unroll
        for (int s = 0; s < 12; ++s) {
            int z = s - 6;
            z += (z < 0) ? n2 : 0;
#pragma unroll
            for (int i = 0; i < C; ++i)
                Q[s][i] = valid[i] ? pb[int64_t(z) * P + col[i]] : T2{0, 0};
        }
        for (int zo = 0; zo < n2; ++zo) {
            int zl = zo + 6;
            zl -= (zl >= n2) ? n2 : 0;
#pragma unroll
            for (int i = 0; i < C; ++i)
                Q[12][i] = valid[i] ? pb[int64_t(zl) * P + col[i]] : T2{0, 0};
            T2* L = lds + (zo & 1) * P;
#pragma unroll
            for (int i = 0; i < C; ++i)
                if (valid[i]) L[col[i]] = Q[6][i];
            __syncthreads();
#pragma unroll
            for (int i = 0; i < C; ++i) {
                if (!valid[i]) continue;
                const int64_t idx = int64_t(zo) * P + col[i];
                const T diag = T(a.cw[0] + a.vloc[idx] - eps_n);
                const T2 q = apply_a<T, T2, C>(a, L, Q, i, cx[i], cy[i], diag, om);
                const T2 c = Q[6][i];
                T2 rv = r[idx];
                rv.x -= ar * q.x - ai * q.y;
                rv.y -= ar * q.y + ai * q.x;
                r[idx] = rv;
                if constexpr (XC) {
                    T2* xp = reinterpret_cast<T2*>(a.x) + off;
                    T2 xv = first ? T2{0, 0} : xp[idx];
                    xv.x += ar * c.x - ai * c.y;
                    xv.y += ar * c.y + ai * c.x;
                    xp[idx] = xv;
                } else {
                    T* xp = reinterpret_cast<T*>(a.x) + off;
                    T xv = first ? T(0) : xp[idx];
                    xv += ar * c.x - ai * c.y;
                    xp[idx] = xv;
                }
                acc2[0] += double(rv.x) * rv.x - double(rv.y) * rv.y;
                acc2[1] += 2.0 * double(rv.x) * rv.y;
                acc2[2] += double(rv.x) * rv.x + double(rv.y) * rv.y;
            }
#pragma unroll
            for (int s = 0; s < 12; ++s)
#pragma unroll
                for (int i = 0; i < C; ++i) Q[s][i] = Q[s + 1][i];
        }
        wg_reduce<3>(acc2, red);
        if (zero_rhs) {
            done = true;  // x = 0 was written by the sweep (alpha = 0, first)
        } else if (breakdown) {
            st = 2;
            done = true;
        } else if (acc2[2] <= a.tol2 * bb) {
            done = true;
        } else if (it >= a.max_iter) {
            st = 1;
            done = true;
        } else {
            const double n2r = acc2[0] * acc2[0] + acc2[1] * acc2[1];
            if (!(n2r > a.bd_tol * a.bd_tol * acc2[2] * acc2[2])) {
                st = 2;
                done = true;
            } else {
                const double rr = rho_re * rho_re + rho_im * rho_im;
                beta_re = (acc2[0] * rho_re + acc2[1] * rho_im) / rr;
                beta_im = (acc2[1] * rho_re - acc2[0] * rho_im) / rr;
                rho_re = acc2[0];
                rho_im = acc2[1];
                T2* t = pa;
                pa = pb;
                pb = t;
            }
        }
    }
    if (tid == 0) {
        a.iters[sys] = it;
        a.status[sys] = st;
    }
}

struct Variant {
    int C;
    int bsmax;
};

template <typename T, int C, int BSMAX, bool XC>
hipError_t launch_variant(const CocgArgs& args, int bs, int nsys, size_t shmem, hipStream_t s) {
    auto fn = cocg_wg<T, C, BSMAX, XC>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(shmem));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fn, dim3(nsys), dim3(bs), shmem, s, args);
    return hipGetLastError();
}

template <typename T, bool XC>
hipError_t dispatch(const CocgArgs& args, int C, int bs, int nsys, size_t shmem,
                    hipStream_t s) {
    const int bsmax = bs <= 256 ? 256 : bs <= 512 ? 512 : bs <= 768 ? 768 : 1024;
#define RPA_CASE(CC, BM)                                           \
    if (C == CC && bsmax == BM)                                    \
        return launch_variant<T, CC, BM, XC>(args, bs, nsys, shmem, s);
    RPA_CASE(1, 256) RPA_CASE(1, 512) RPA_CASE(1, 768) RPA_CASE(1, 1024)
    RPA_CASE(2, 256) RPA_CASE(2, 512) RPA_CASE(2, 768) RPA_CASE(2, 1024)
    RPA_CASE(3, 256) RPA_CASE(3, 512) RPA_CASE(3, 768) RPA_CASE(3, 1024)
    RPA_CASE(4, 256) RPA_CASE(4, 512) RPA_CASE(4, 768) RPA_CASE(4, 1024)
#undef RPA_CASE
    return hipErrorInvalidConfiguration;
}

}  // namespace

// Choose columns-per-thread C and block size: smallest idle fraction, preferring a
// register footprint that fits without spilling (queue of 13 complex values per column).
static void choose_shape(int P, bool fp32, int* C_out, int* bs_out) {
    int bestC = 4, bestBS = 1024;
    double best = 1e30;
    for (int C = 1; C <= 4; ++C) {
        int bs = ((P + C - 1) / C + 63) / 64 * 64;
        if (bs > 1024) continue;
        const int waves_per_simd = (bs / 64 + 3) / 4;
        const int budget = 512 / waves_per_simd;
        const int need = (fp32 ? 26 : 52) * C + 48;
        const double idle = double(bs * C - P) / double(bs * C);
        const double cost = idle + (need > budget ? 1.0 + 0.01 * (need - budget) : 0.0);
        if (cost < best - 1e-12) {
            best = cost;
            bestC = C;
            bestBS = bs;
        }
    }
    *C_out = bestC;
    *bs_out = bestBS;
}

hipError_t launch_cocg(const CocgLaunch& L, hipStream_t s) {
    if (L.nsys <= 0) return hipSuccess;
    CocgArgs a{};
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
    a.tol2 = L.tol * L.tol;
    a.max_iter = L.max_iter;
    a.bd_tol = L.fp32 ? 1e-6 : 1e-14;
    a.nd = L.g.nd();
    a.r = L.r;
    a.pa = L.pa;
    a.pb = L.pb;
    a.x = L.x;
    a.iters = L.iters;
    a.status = L.status;
    int C, bs;
    choose_shape(a.P, L.fp32, &C, &bs);
    const size_t t2 = L.fp32 ? sizeof(float2) : sizeof(double2);
    const size_t shmem = 2 * size_t(a.P) * t2 + 16 * 8 * sizeof(double);
    if (L.fp32) {
        return L.x_complex ? dispatch<float, true>(a, C, bs, L.nsys, shmem, s)
                           : dispatch<float, false>(a, C, bs, L.nsys, shmem, s);
    }
    return L.x_complex ? dispatch<double, true>(a, C, bs, L.nsys, shmem, s)
                       : dispatch<double, false>(a, C, bs, L.nsys, shmem, s);
}

}  // namespace rpa
