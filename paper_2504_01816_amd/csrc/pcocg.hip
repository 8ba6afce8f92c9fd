// Preconditioned COCG for the Sternheimer systems (H - eps_n - i omega) x = b with the
// Kronecker shifted-Laplacian preconditioner K_s^{-1}, K_s = -1/2 Lap_h + sigma_n - i omega
// (the Laplacian-based preconditioning through the Kronecker product formalism that Sec. 3
// offers as an alternative to the projector-based initial guess).  K_s is complex
// symmetric, so the iteration keeps COCG's unconjugated bilinear form:
//
//     r = b, z = M r, p = z, rho = r^T z
//     repeat:  q = A p; alpha = rho / p^T q; x += alpha p; r -= alpha q   (pc_step)
//              stop when ||r|| <= tol ||b||
//              z = M r                                                  (Kronecker passes)
//              rho' = r^T z; p = z + (rho'/rho) p                       (pc_rz)
//
// Design: the preconditioner needs whole-vector transforms along every axis, which do not
// fit the register-resident z-march of the plain COCG kernel, so each iteration is a few
// batched launches driven by the host: the step q = A p with the x and r updates runs one
// workgroup per system on the plain kernel's z-march (pc_step_wg; pc_step, which gathers
// the 36 neighbours through the caches, where no march shape fits); pc_rz does r^T z and the
// p update; reductions are workgroup-local and in a fixed order.  z = M r is three
// LDS-staged passes (x-y planes forward, z pencils with the diagonal scale, x-y planes
// inverse) over all systems at once for short axes, else 3 + 3 Kronecker GEMM passes with a
// diagonal scale.  Every thread touches the same points in both loops of a kernel, so a
// value a thread writes is read back only by itself.  Converged systems drop out of the
// per-system kernels; the host tests for the end every few iterations.
// Slots: the systems are placed in slots t = 0 .. nsys-1 in the dispatch order (expected
// longest solve first), so the systems still iterating gather in a prefix of the slots and
// the preconditioner passes run on that prefix only.
// Layout: r, p, z, q as N_d x 2 nsys real columns (real, imaginary part of slot t in columns
// 2t, 2t+1), rho, b2, active and the preconditioner shifts per slot; x, the right-hand
// sides, iteration counts and statuses per system, x and b complex interleaved, nsys x N_d.
// The same buffers and kernels serve block COCG (options.cocg_block, the block variant of the
// solver that Sec. 3 names with the preconditioner): the step stores q only and block
// kernels, one workgroup per block of slots, take the place of the scalar recurrences.
#include <cstdlib>
#include <cstring>
#include <vector>

#include "cocg_kernel.h"
#include "internal.h"

namespace rpa {
namespace {

constexpr int PB = 256;
constexpr int kCheckEvery = 8;   // iterations between tests for the end

struct PcArgs {
    int n0, n1, n2, periodic;
    int64_t nd;
    double cw[7];   // cw[k] = -1/2 w_k / h^2 (k >= 1); cw[0] = -1/2 * 3 w_0 / h^2
    const double* vloc;
    const double* eps;
    const double* omega_v;
    int ns;
    double tol2, bd_tol;
    int max_iter;
    double *r, *p, *z, *q;
    double2* x;
    const double2* rhs;
    double2* rho;
    double* b2;
    int *active, *iters, *status;
    const int* order;   // slot t holds system order[t]
    int qonly;          // the step stores q = A p and stops (block COCG)
    const int* boff;    // block COCG: slots of block b are boff[b] .. boff[b+1]-1
    int* split;         // block COCG, per slot (block b at boff[b]): state + 4 * live mask at
                        // the last direction step; state 0 block, 1 split with a restart
                        // pending, 2 split (single-vector iterations)
};

// Sum of NV values over the workgroup, in a fixed order (wave butterfly, then waves in order);
// every thread receives the sums.
template <int NV>
__device__ void pc_reduce(double (&v)[NV], double* red) {
    for (int o = 32; o > 0; o >>= 1)
        for (int k = 0; k < NV; ++k) v[k] += __shfl_xor(v[k], o, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane == 0)
        for (int k = 0; k < NV; ++k) red[wave * NV + k] = v[k];
    __syncthreads();
    for (int k = 0; k < NV; ++k) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += red[w * NV + k];
        v[k] = s;
    }
    __syncthreads();
}

// r = b (split), x = 0, |b|^2; systems with b = 0 are done (x = 0).
__global__ __launch_bounds__(PB) void pc_start(PcArgs a) {
    __shared__ double red[(PB / 64) * 1];
    const int s = blockIdx.x, sys = a.order[s];
    const int64_t nd = a.nd;
    const double2* b = a.rhs + int64_t(sys) * nd;
    double* rr = a.r + nd * (2 * int64_t(s));
    double* ri = rr + nd;
    double2* x = a.x + int64_t(sys) * nd;
    double acc[1] = {0.0};
    for (int64_t i = threadIdx.x; i < nd; i += PB) {
        const double2 v = b[i];
        rr[i] = v.x;
        ri[i] = v.y;
        x[i] = double2{0.0, 0.0};
        acc[0] += v.x * v.x + v.y * v.y;
    }
    pc_reduce<1>(acc, red);
    if (threadIdx.x == 0) {
        a.b2[s] = acc[0];
        a.active[s] = acc[0] > 0.0 ? 1 : 0;
        a.iters[sys] = 0;
        a.status[sys] = 0;
        if (a.split) a.split[s] = 0;
    }
}

// One neighbour value of the split vector v at (x + dx, y + dy, z + dz); 0 beyond the walls of
// an isolated box.
__device__ __forceinline__ double nb(const double* v, const PcArgs& a, int x, int y, int z) {
    if (a.periodic) {
        x += (x < 0) ? a.n0 : 0;
        x -= (x >= a.n0) ? a.n0 : 0;
        y += (y < 0) ? a.n1 : 0;
        y -= (y >= a.n1) ? a.n1 : 0;
        z += (z < 0) ? a.n2 : 0;
        z -= (z >= a.n2) ? a.n2 : 0;
    } else if (x < 0 || x >= a.n0 || y < 0 || y >= a.n1 || z < 0 || z >= a.n2) {
        return 0.0;
    }
    return v[x + int64_t(a.n0) * (y + int64_t(a.n1) * z)];
}

// q = A p, sigma = p^T q; alpha = rho / sigma; x += alpha p; r -= alpha q; convergence test.
__global__ __launch_bounds__(PB) void pc_step(PcArgs a, int it) {
    __shared__ double red[(PB / 64) * 4];
    const int s = blockIdx.x;
    if (!a.active[s]) return;
    const int sys = a.order[s];
    const int64_t nd = a.nd;
    const double eps = a.eps[sys % a.ns], om = a.omega_v[sys / a.ns];
    const double* pr = a.p + nd * (2 * int64_t(s));
    const double* pi = pr + nd;
    double* qr = a.q + nd * (2 * int64_t(s));
    double* qi = qr + nd;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};   // sigma re/im, |p|^2, |q|^2
    for (int64_t i = threadIdx.x; i < nd; i += PB) {
        const int x = int(i % a.n0), y = int((i / a.n0) % a.n1), z = int(i / (int64_t(a.n0) * a.n1));
        double sr = 0.0, si = 0.0;
        for (int k = 1; k <= 6; ++k) {
            const double tr = nb(pr, a, x + k, y, z) + nb(pr, a, x - k, y, z) +
                              nb(pr, a, x, y + k, z) + nb(pr, a, x, y - k, z) +
                              nb(pr, a, x, y, z + k) + nb(pr, a, x, y, z - k);
            const double ti = nb(pi, a, x + k, y, z) + nb(pi, a, x - k, y, z) +
                              nb(pi, a, x, y + k, z) + nb(pi, a, x, y - k, z) +
                              nb(pi, a, x, y, z + k) + nb(pi, a, x, y, z - k);
            sr += a.cw[k] * tr;
            si += a.cw[k] * ti;
        }
        const double d = a.cw[0] + a.vloc[i] - eps;
        const double p0r = pr[i], p0i = pi[i];
        // (V - eps - i omega) p: real part d p_r + omega p_i, imaginary part d p_i - omega p_r
        const double vr = sr + d * p0r + om * p0i;
        const double vi = si + d * p0i - om * p0r;
        qr[i] = vr;
        qi[i] = vi;
        acc[0] += p0r * vr - p0i * vi;
        acc[1] += p0r * vi + p0i * vr;
        acc[2] += p0r * p0r + p0i * p0i;
        acc[3] += vr * vr + vi * vi;
    }
    if (a.qonly) return;
    pc_reduce<4>(acc, red);
    const double s2 = acc[0] * acc[0] + acc[1] * acc[1];
    if (!(s2 > a.bd_tol * a.bd_tol * acc[2] * acc[3])) {   // vanishing p^T q: breakdown
        if (threadIdx.x == 0) {
            a.iters[sys] = it;
            a.status[sys] = 2;
            a.active[s] = 0;
        }
        return;
    }
    const double2 rho = a.rho[s];
    const double ar = (rho.x * acc[0] + rho.y * acc[1]) / s2;
    const double ai = (rho.y * acc[0] - rho.x * acc[1]) / s2;
    double* rr = a.r + nd * (2 * int64_t(s));
    double* ri = rr + nd;
    double2* xs = a.x + int64_t(sys) * nd;
    double acc2[1] = {0.0};
    for (int64_t i = threadIdx.x; i < nd; i += PB) {
        const double p0r = pr[i], p0i = pi[i], q0r = qr[i], q0i = qi[i];
        double2 xv = xs[i];
        xv.x += ar * p0r - ai * p0i;
        xv.y += ar * p0i + ai * p0r;
        xs[i] = xv;
        const double nr = rr[i] - (ar * q0r - ai * q0i);
        const double ni = ri[i] - (ar * q0i + ai * q0r);
        rr[i] = nr;
        ri[i] = ni;
        acc2[0] += nr * nr + ni * ni;
    }
    pc_reduce<1>(acc2, red);
    if (threadIdx.x == 0) {
        a.iters[sys] = it;
        if (acc2[0] <= a.tol2 * a.b2[s]) {
            a.active[s] = 0;
        } else if (it >= a.max_iter) {
            a.status[sys] = 1;
            a.active[s] = 0;
        }
    }
}

constexpr int RZB = 1024;   // threads of pc_rz (a streaming pass: more waves in flight)

// rho' = r^T z; first: p = z, else p = z + (rho'/rho) p; rho = rho'.
__global__ __launch_bounds__(RZB) void pc_rz(PcArgs a, int first) {
    __shared__ double red[(RZB / 64) * 4];
    const int s = blockIdx.x;
    if (!a.active[s]) return;
    const int64_t nd = a.nd;
    const double* rr = a.r + nd * (2 * int64_t(s));
    const double* ri = rr + nd;
    const double* zr = a.z + nd * (2 * int64_t(s));
    const double* zi = zr + nd;
    double* pr = a.p + nd * (2 * int64_t(s));
    double* pi = pr + nd;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};   // rho' re/im, |r|^2, |z|^2
    for (int64_t i = threadIdx.x; i < nd; i += RZB) {
        const double a0 = rr[i], a1 = ri[i], c0 = zr[i], c1 = zi[i];
        acc[0] += a0 * c0 - a1 * c1;
        acc[1] += a0 * c1 + a1 * c0;
        acc[2] += a0 * a0 + a1 * a1;
        acc[3] += c0 * c0 + c1 * c1;
    }
    pc_reduce<4>(acc, red);
    const double n2 = acc[0] * acc[0] + acc[1] * acc[1];
    if (!(n2 > a.bd_tol * a.bd_tol * acc[2] * acc[3])) {   // vanishing r^T z: breakdown
        if (threadIdx.x == 0) {
            a.status[a.order[s]] = 2;
            a.active[s] = 0;
        }
        return;
    }
    double br = 0.0, bi = 0.0;
    if (!first) {
        const double2 rho = a.rho[s];
        const double rr2 = rho.x * rho.x + rho.y * rho.y;
        br = (acc[0] * rho.x + acc[1] * rho.y) / rr2;
        bi = (acc[1] * rho.x - acc[0] * rho.y) / rr2;
    }
    for (int64_t i = threadIdx.x; i < nd; i += RZB) {
        const double o0 = first ? 0.0 : pr[i], o1 = first ? 0.0 : pi[i];
        pr[i] = zr[i] + br * o0 - bi * o1;
        pi[i] = zi[i] + br * o1 + bi * o0;
    }
    if (threadIdx.x == 0) a.rho[s] = double2{acc[0], acc[1]};
}

// ------------------------------------------------------------------ block COCG
// Block COCG over the systems of one orbital and one frequency (one matrix A, one K^{-1}),
// one workgroup per block of w <= kMaxBlockWidth consecutive slots.  The columns still
// iterating form the live set L (active flags); a converged column is frozen and every
// w x w quantity is taken on L:
//     q = A p on the live slots                                   (step kernel, q only)
//     alpha = (P^T Q)^{-1} rho; X += P alpha; R -= Q alpha; tests   (bc_update)
//     Z = M R on the live slots                                   (preconditioner passes)
//     rho' = R^T Z; beta = rho^{-1} rho'; P = Z + P beta; rho = rho' (bc_dir)
// The w x w matrices are reduced in a fixed order and solved by one thread; rho is kept per
// block as rows of kMaxBlockWidth entries, row c at slot s0 + c.  When columns converge the
// block restarts on the rest (beta = 0: the kept directions are not conjugate within the
// smaller block).  A block whose residual columns lose rank (a small solve with a scaled pivot
// <= kSplitTol) splits: its live columns go on as single-vector iterations (diagonal alpha
// and beta), restarting with p = z at the next direction step.
constexpr int LDW = kMaxBlockWidth;
// Pivot threshold of the scaled small solves below which a block counts as rank deficient and
// splits (a condition number beyond ~1e3 after scaling; 1e-2 splits blocks that converge).
constexpr double kSplitTol = 1e-3;
constexpr int BPB = 1024;   // threads per block-COCG workgroup (one block per workgroup)

__device__ __forceinline__ double2 cmul(double2 u, double2 v) {
    return double2{u.x * v.x - u.y * v.y, u.x * v.y + u.y * v.x};
}
__device__ __forceinline__ double2 cdiv(double2 u, double2 v) {
    const double d = v.x * v.x + v.y * v.y;
    return double2{(u.x * v.x + u.y * v.y) / d, (u.y * v.x - u.x * v.y) / d};
}
__device__ __forceinline__ double cmod(double2 u) { return hypot(u.x, u.y); }

// Y <- M^{-1} Y for the n x n leading parts of row-major LDW x LDW arrays (M is destroyed):
// rows, then columns of M scaled to a largest modulus of one (the entries scale with the
// residual norms of their columns, which differ by up to the tolerance ratio), Gaussian
// elimination with partial pivoting (first row of largest modulus), back substitution and the
// column scales.  false when a row or column is zero or a pivot's modulus is <= bd_tol.
// cs: LDW doubles of LDS for the column scales.
__device__ bool small_solve(double2* M, double2* Y, int n, double bd_tol, double* cs) {
    for (int i = 0; i < n; ++i) {
        double m = 0.0;
        for (int j = 0; j < n; ++j) m = fmax(m, cmod(M[i * LDW + j]));
        if (!(m > 0.0)) return false;
        for (int j = 0; j < n; ++j) {
            M[i * LDW + j].x /= m;
            M[i * LDW + j].y /= m;
            Y[i * LDW + j].x /= m;
            Y[i * LDW + j].y /= m;
        }
    }
    for (int j = 0; j < n; ++j) {
        double m = 0.0;
        for (int i = 0; i < n; ++i) m = fmax(m, cmod(M[i * LDW + j]));
        if (!(m > 0.0)) return false;
        for (int i = 0; i < n; ++i) {
            M[i * LDW + j].x /= m;
            M[i * LDW + j].y /= m;
        }
        cs[j] = m;
    }
    for (int k = 0; k < n; ++k) {
        int piv = k;
        double best = cmod(M[k * LDW + k]);
        for (int i = k + 1; i < n; ++i) {
            const double m = cmod(M[i * LDW + k]);
            if (m > best) {
                best = m;
                piv = i;
            }
        }
        if (!(best > bd_tol)) return false;
        if (piv != k)
            for (int j = 0; j < n; ++j) {
                const double2 t = M[k * LDW + j];
                M[k * LDW + j] = M[piv * LDW + j];
                M[piv * LDW + j] = t;
                const double2 u = Y[k * LDW + j];
                Y[k * LDW + j] = Y[piv * LDW + j];
                Y[piv * LDW + j] = u;
            }
        for (int i = k + 1; i < n; ++i) {
            const double2 f = cdiv(M[i * LDW + k], M[k * LDW + k]);
            for (int j = k; j < n; ++j) {
                const double2 t = cmul(f, M[k * LDW + j]);
                M[i * LDW + j].x -= t.x;
                M[i * LDW + j].y -= t.y;
            }
            for (int j = 0; j < n; ++j) {
                const double2 t = cmul(f, Y[k * LDW + j]);
                Y[i * LDW + j].x -= t.x;
                Y[i * LDW + j].y -= t.y;
            }
        }
    }
    for (int k = n - 1; k >= 0; --k)
        for (int j = 0; j < n; ++j) {
            double2 acc = Y[k * LDW + j];
            for (int l = k + 1; l < n; ++l) {
                const double2 t = cmul(M[k * LDW + l], Y[l * LDW + j]);
                acc.x -= t.x;
                acc.y -= t.y;
            }
            Y[k * LDW + j] = cdiv(acc, M[k * LDW + k]);
        }
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j) {
            Y[k * LDW + j].x /= cs[k];
            Y[k * LDW + j].y /= cs[k];
        }
    return true;
}

// Live mask of the block at slots s0 .. s0+w-1 (bit c: slot s0 + c still iterating).
__device__ __forceinline__ unsigned block_live(const PcArgs& a, int s0, int w) {
    unsigned m = 0;
    for (int c = 0; c < w; ++c)
        if (a.active[s0 + c]) m |= 1u << c;
    return m;
}

// Rows of the block Gram matrices reduced per pass (bounds the accumulator registers).
template <int SM>
constexpr int gram_rows() { return SM < 4 ? SM : 4; }

// out[k] = sum over the workgroup of v[k] (LDS), in a fixed order: a butterfly in every wave,
// one value at a time (a scheduling barrier keeps one value's shuffles in flight), then the
// waves in order.  Ends with a barrier.
template <int NV>
__device__ void gram_reduce(const double (&v)[NV], double* red, double* out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double x = v[k];
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
        if (lane == 0) red[wave * NV + k] = x;
        __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double t = 0.0;
        for (int w = 0; w < nw; ++w) t += red[w * NV + threadIdx.x];
        out[threadIdx.x] = t;
    }
    __syncthreads();
}

// gm[2 (c SM + d) + {0, 1}] = u_c^T v_d (unconjugated) over the live pairs (LDS), reduced over
// the workgroup in a fixed order, rows in passes of gram_rows.
template <int SM>
__device__ void block_gram(const double* u, const double* v, int s0, unsigned live, int64_t nd,
                           double* gm, double* red) {
    constexpr int RB = gram_rows<SM>();
#pragma unroll 1
    for (int c0 = 0; c0 < SM; c0 += RB) {
        if (!(live >> c0 & ((1u << RB) - 1u))) continue;
        double acc[2 * RB * SM];
        for (int k = 0; k < 2 * RB * SM; ++k) acc[k] = 0.0;
#pragma unroll 1
        for (int64_t i = threadIdx.x; i < nd; i += BPB) {
            double2 vv[SM];
#pragma unroll
            for (int d = 0; d < SM; ++d)
                if (live >> d & 1u) {
                    const double* vd = v + nd * (2 * int64_t(s0 + d));
                    vv[d] = double2{vd[i], vd[i + nd]};
                }
#pragma unroll
            for (int cc = 0; cc < RB; ++cc) {
                if (!(live >> (c0 + cc) & 1u)) continue;
                const double* uc = u + nd * (2 * int64_t(s0 + c0 + cc));
                const double2 uu{uc[i], uc[i + nd]};
#pragma unroll
                for (int d = 0; d < SM; ++d)
                    if (live >> d & 1u) {
                        acc[2 * (cc * SM + d)] += uu.x * vv[d].x - uu.y * vv[d].y;
                        acc[2 * (cc * SM + d) + 1] += uu.x * vv[d].y + uu.y * vv[d].x;
                    }
            }
        }
        gram_reduce<2 * RB * SM>(acc, red, gm + 2 * c0 * SM);
    }
}

// Compacts the live rows and columns of an SM x SM matrix held as (re, im) pairs into the
// leading nl x nl part of dst.
template <int SM>
__device__ int compact_acc(const double* acc, unsigned live, double2* dst) {
    int r = 0;
    for (int c = 0; c < SM; ++c) {
        if (!(live >> c & 1u)) continue;
        int q = 0;
        for (int d = 0; d < SM; ++d) {
            if (!(live >> d & 1u)) continue;
            dst[r * LDW + q] = double2{acc[2 * (c * SM + d)], acc[2 * (c * SM + d) + 1]};
            ++q;
        }
        ++r;
    }
    return r;
}

// Scatters the leading nl x nl part of src (live order) to the full w x w layout of dst
// (zero outside the live rows and columns).
__device__ void expand_live(const double2* src, unsigned live, int w, double2* dst) {
    int r = 0;
    for (int c = 0; c < LDW; ++c) {
        const bool lc = c < w && (live >> c & 1u);
        int q = 0;
        for (int d = 0; d < LDW; ++d) {
            const bool ld = d < w && (live >> d & 1u);
            dst[c * LDW + d] = (lc && ld) ? src[r * LDW + q] : double2{0.0, 0.0};
            q += ld ? 1 : 0;
        }
        r += lc ? 1 : 0;
    }
}

// G = P^T Q on L; alpha = G^{-1} rho; X += P alpha; R -= Q alpha; convergence and cap tests.
template <int SM>
__global__ __launch_bounds__(BPB) void bc_update(PcArgs a, int it) {
    __shared__ double red[(BPB / 64) * 2 * gram_rows<SM>() * SM];
    __shared__ double acc[2 * SM * SM];
    __shared__ double2 G[LDW * LDW], Y[LDW * LDW], AL[LDW * LDW];
    __shared__ double cs[LDW];
    const int s0 = a.boff[blockIdx.x], w = a.boff[blockIdx.x + 1] - s0;
    const unsigned live = block_live(a, s0, w);
    if (!live) return;
    const int64_t nd = a.nd;
    const int sp = a.split[s0] & 3;
    block_gram<SM>(a.p, a.q, s0, live, nd, acc, red);
    if (threadIdx.x == 0) {
        bool ok = false;
        if (sp == 0) {
            const int nl = compact_acc<SM>(acc, live, G);
            int r = 0;
            for (int c = 0; c < w; ++c) {
                if (!(live >> c & 1u)) continue;
                int q = 0;
                for (int d = 0; d < w; ++d)
                    if (live >> d & 1u) Y[r * LDW + q++] = a.rho[(s0 + c) * LDW + d];
                ++r;
            }
            ok = small_solve(G, Y, nl, kSplitTol, cs);
            if (ok) expand_live(Y, live, w, AL);
            else a.split[s0] = (a.split[s0] & ~3) | 1;
        }
        if (!ok) {
            // split: alpha_c = rho_cc / (p_c^T q_c); a zero denominator breaks the column down
            for (int e = 0; e < LDW * LDW; ++e) AL[e] = double2{0.0, 0.0};
            for (int c = 0; c < SM; ++c) {
                if (!(live >> c & 1u)) continue;
                const double2 g{acc[2 * (c * SM + c)], acc[2 * (c * SM + c) + 1]};
                if (g.x == 0.0 && g.y == 0.0) {
                    a.status[a.order[s0 + c]] = 2;
                    a.active[s0 + c] = 0;
                } else {
                    AL[c * LDW + c] = cdiv(a.rho[(s0 + c) * LDW + c], g);
                }
            }
        }
        for (int c = 0; c < w; ++c)
            if (live >> c & 1u) a.iters[a.order[s0 + c]] = it;
    }
    __syncthreads();
    double nrm[SM];
    for (int c = 0; c < SM; ++c) nrm[c] = 0.0;
    for (int64_t i = threadIdx.x; i < nd; i += BPB) {
        // an offset the compiler cannot see through keeps the coefficient reads (broadcast
        // LDS loads) inside the loop instead of holding SM x SM of them in registers
        int o = 0;
        asm volatile("" : "+v"(o));
        double2 pv[SM], qv[SM];
#pragma unroll
        for (int k = 0; k < SM; ++k)
            if (live >> k & 1u) {
                const double* pk = a.p + nd * (2 * int64_t(s0 + k));
                const double* qk = a.q + nd * (2 * int64_t(s0 + k));
                pv[k] = double2{pk[i], pk[i + nd]};
                qv[k] = double2{qk[i], qk[i + nd]};
            }
#pragma unroll
        for (int c = 0; c < SM; ++c) {
            if (!(live >> c & 1u)) continue;
            double2 dx{0.0, 0.0}, dr{0.0, 0.0};
#pragma unroll
            for (int k = 0; k < SM; ++k)
                if (live >> k & 1u) {
                    const double2 al = AL[o + k * LDW + c];
                    const double2 t = cmul(pv[k], al), u = cmul(qv[k], al);
                    dx.x += t.x;
                    dx.y += t.y;
                    dr.x += u.x;
                    dr.y += u.y;
                }
            double2* xc = a.x + int64_t(a.order[s0 + c]) * nd;
            double2 xv = xc[i];
            xv.x += dx.x;
            xv.y += dx.y;
            xc[i] = xv;
            double* rc = a.r + nd * (2 * int64_t(s0 + c));
            const double nr = rc[i] - dr.x, ni = rc[i + nd] - dr.y;
            rc[i] = nr;
            rc[i + nd] = ni;
            nrm[c] += nr * nr + ni * ni;
        }
    }
    pc_reduce<SM>(nrm, red);
    if (threadIdx.x == 0)
        for (int c = 0; c < w; ++c) {
            if (!(live >> c & 1u) || !a.active[s0 + c]) continue;   // broken down above
            if (nrm[c] <= a.tol2 * a.b2[s0 + c]) {
                a.active[s0 + c] = 0;
            } else if (it >= a.max_iter) {
                a.status[a.order[s0 + c]] = 1;
                a.active[s0 + c] = 0;
            }
        }
}

// rho' = R^T Z on L; first: P = Z; else beta = rho^{-1} rho', P = Z + P beta; rho = rho'.
// A split block restarts (beta = 0) once, then takes beta_c = rho'_cc / rho_cc.
template <int SM>
__global__ __launch_bounds__(BPB) void bc_dir(PcArgs a, int first) {
    __shared__ double red[(BPB / 64) * 2 * gram_rows<SM>() * SM];
    __shared__ double acc[2 * SM * SM];
    __shared__ double2 G[LDW * LDW], Y[LDW * LDW], BE[LDW * LDW];
    __shared__ double cs[LDW];
    const int s0 = a.boff[blockIdx.x], w = a.boff[blockIdx.x + 1] - s0;
    const unsigned live = block_live(a, s0, w);
    if (!live) return;
    const int64_t nd = a.nd;
    const int sv = a.split[s0], sp = sv & 3;
    const bool shrank = (unsigned(sv >> 2) & ~live) != 0u;   // columns converged since
    block_gram<SM>(a.r, a.z, s0, live, nd, acc, red);
    if (threadIdx.x == 0 && !first) {
        bool ok = false;
        int state = sp;
        if (sp == 0 && shrank) {
            for (int e = 0; e < LDW * LDW; ++e) BE[e] = double2{0.0, 0.0};   // restart
            ok = true;
        } else if (sp == 0) {
            const int nl = compact_acc<SM>(acc, live, Y);
            int r = 0;
            for (int c = 0; c < w; ++c) {
                if (!(live >> c & 1u)) continue;
                int q = 0;
                for (int d = 0; d < w; ++d)
                    if (live >> d & 1u) G[r * LDW + q++] = a.rho[(s0 + c) * LDW + d];
                ++r;
            }
            ok = small_solve(G, Y, nl, kSplitTol, cs);
            if (ok) expand_live(Y, live, w, BE);
        }
        if (!ok) {
            for (int e = 0; e < LDW * LDW; ++e) BE[e] = double2{0.0, 0.0};
            if (sp == 2) {
                // split: beta_c = rho'_cc / rho_cc; a zero rho_cc breaks the column down
                for (int c = 0; c < SM; ++c) {
                    if (!(live >> c & 1u)) continue;
                    const double2 d = a.rho[(s0 + c) * LDW + c];
                    if (d.x == 0.0 && d.y == 0.0) {
                        a.status[a.order[s0 + c]] = 2;
                        a.active[s0 + c] = 0;
                    } else {
                        BE[c * LDW + c] = cdiv(double2{acc[2 * (c * SM + c)],
                                                       acc[2 * (c * SM + c) + 1]}, d);
                    }
                }
            } else {
                state = 2;   // restart: p = z
            }
        }
        a.split[s0] = state | int(live << 2);
    }
    if (threadIdx.x == 0 && first) a.split[s0] = int(live << 2);
    if (threadIdx.x == 0)
        for (int c = 0; c < SM; ++c)
            for (int d = 0; d < SM; ++d)
                if ((live >> c & 1u) && (live >> d & 1u))
                    a.rho[(s0 + c) * LDW + d] =
                        double2{acc[2 * (c * SM + d)], acc[2 * (c * SM + d) + 1]};
    __syncthreads();
    for (int64_t i = threadIdx.x; i < nd; i += BPB) {
        int o = 0;   // keeps the coefficient reads inside the loop (as in bc_update)
        asm volatile("" : "+v"(o));
        double2 pv[SM];
        if (!first) {
#pragma unroll
            for (int k = 0; k < SM; ++k)
                if (live >> k & 1u) {
                    const double* pk = a.p + nd * (2 * int64_t(s0 + k));
                    pv[k] = double2{pk[i], pk[i + nd]};
                }
        }
#pragma unroll
        for (int c = 0; c < SM; ++c) {
            if (!(live >> c & 1u)) continue;
            const double* zc = a.z + nd * (2 * int64_t(s0 + c));
            double2 v{zc[i], zc[i + nd]};
            if (!first) {
#pragma unroll
                for (int k = 0; k < SM; ++k)
                    if (live >> k & 1u) {
                        const double2 t = cmul(pv[k], BE[o + k * LDW + c]);
                        v.x += t.x;
                        v.y += t.y;
                    }
            }
            double* pc = a.p + nd * (2 * int64_t(s0 + c));
            pc[i] = v.x;
            pc[i + nd] = v.y;
        }
    }
}

// ------------------------------------------------------------------ fused preconditioner
// z = K^{-1} r in three passes instead of six GEMM passes and a scale pass: forward x and y
// transforms of one z-plane of one system in LDS; forward z transform, diagonal scale and
// inverse z transform of 64 z-pencils in LDS (results of the forward transform in
// registers); inverse y and x transforms per plane.  The dense 1D transforms cost n LDS
// multiply-adds per point and axis, so the fused passes beat the MFMA GEMM passes only for
// short axes (measured on the whole solve: 1.25x faster than the GEMM passes at 24^3, before
// the forward x basis was stored transposed, which took the solve from 368 to 313 ms; 118
// against 70 s at 48^3 after it); used for n0, n1, n2 <= 32.
constexpr int kFusedMaxXY = 32;
constexpr int kFusedMaxZ = 32;
constexpr int kPencils = 64;
constexpr size_t kMaxLds = 160 * 1024;   // LDS of one workgroup on gfx950
constexpr int ZB = 512;                      // threads of the pencil pass
constexpr int XYB = 512;                     // threads of the plane passes
constexpr int kZr = 64 / (ZB / kPencils);   // z values per thread in the pencil pass (n2 <= 64)

// forward (INV = false): c_(a,b) = sum_(x,y) Ux[x + n0 a] Uy[y + n1 b] f_(x,y); inverse: the
// transposed bases.  grid (n2, systems), in/out: N_d x 2 nsys split columns.
template <bool INV>
__global__ __launch_bounds__(XYB) void pc_xy(const double* in, double* out, int n0, int n1,
                                            int64_t nd, const double* Ux, const double* Uy) {
    extern __shared__ double2 shx[];
    const int P = n0 * n1;
    const int z = blockIdx.x, t = blockIdx.y;
    double2* A = shx;
    double2* B = shx + P;
    double* ux = reinterpret_cast<double*>(shx + 2 * P);
    double* uy = ux + n0 * n0;
    const double* ir = in + nd * (2 * int64_t(t)) + int64_t(z) * P;
    const double* ii = ir + nd;
    for (int i = threadIdx.x; i < P; i += XYB) A[i] = double2{ir[i], ii[i]};
    // x basis stored so that lanes (consecutive a) read consecutive entries: ux[a + n0 k] =
    // U[a + n0 k] for the inverse, U[k + n0 a] (the transpose) for the forward transform
    for (int i = threadIdx.x; i < n0 * n0; i += XYB) {
        const int a = i % n0, k = i / n0;
        ux[i] = INV ? Ux[i] : Ux[k + n0 * a];
    }
    for (int i = threadIdx.x; i < n1 * n1; i += XYB) uy[i] = Uy[i];
    __syncthreads();
    for (int o = threadIdx.x; o < P; o += XYB) {          // along x
        const int y = o / n0, a = o - y * n0;
        double sr = 0.0, si = 0.0;
        for (int k = 0; k < n0; ++k) {
            const double u = ux[a + n0 * k];
            const double2 v = A[y * n0 + k];
            sr += u * v.x;
            si += u * v.y;
        }
        B[o] = double2{sr, si};
    }
    __syncthreads();
    for (int o = threadIdx.x; o < P; o += XYB) {          // along y
        const int b = o / n0, x = o - b * n0;
        double sr = 0.0, si = 0.0;
        for (int k = 0; k < n1; ++k) {
            const double u = INV ? uy[b + n1 * k] : uy[k + n1 * b];
            const double2 v = B[k * n0 + x];
            sr += u * v.x;
            si += u * v.y;
        }
        A[o] = double2{sr, si};
    }
    __syncthreads();
    double* orr = out + nd * (2 * int64_t(t)) + int64_t(z) * P;
    double* oi = orr + nd;
    for (int i = threadIdx.x; i < P; i += XYB) {
        orr[i] = A[i].x;
        oi[i] = A[i].y;
    }
}

// In place on the x-y mode coefficients: forward z transform, division by
// 1/2 (kx + ky + kz) + sigma_t - i omega_t, inverse z transform.  grid (ceil(P/64), systems).
__global__ __launch_bounds__(ZB) void pc_zscale(double* data, int n0, int n1, int n2, int64_t nd,
                                                const double* Uz, const double* kx,
                                                const double* ky, const double* kz,
                                                const double2* kshift) {
    extern __shared__ double2 shz[];
    const int P = n0 * n1;
    const int g0 = blockIdx.x * kPencils, t = blockIdx.y;
    const int j = threadIdx.x % kPencils, cg = threadIdx.x / kPencils, ng = ZB / kPencils;
    double2* Pz = shz;                                          // n2 x 64
    double* uz = reinterpret_cast<double*>(shz + n2 * kPencils);
    double* dr = data + nd * (2 * int64_t(t));
    double* di = dr + nd;
    for (int e = threadIdx.x; e < n2 * kPencils; e += ZB) {
        const int zz = e / kPencils, xy = g0 + (e - zz * kPencils);
        Pz[e] = (xy < P) ? double2{dr[xy + int64_t(P) * zz], di[xy + int64_t(P) * zz]}
                         : double2{0.0, 0.0};
    }
    for (int i = threadIdx.x; i < n2 * n2; i += ZB) uz[i] = Uz[i];
    __syncthreads();
    double2 acc[kZr];
#pragma unroll
    for (int k = 0; k < kZr; ++k) {
        const int c = cg + ng * k;
        double sr = 0.0, si = 0.0;
        if (c < n2) {
            for (int zz = 0; zz < n2; ++zz) {
                const double u = uz[zz + n2 * c];
                const double2 v = Pz[zz * kPencils + j];
                sr += u * v.x;
                si += u * v.y;
            }
        }
        acc[k] = double2{sr, si};
    }
    __syncthreads();                                            // every read of Pz done
    const int xy = g0 + j;
    const int a = xy % n0, b = (xy / n0) % n1;
    const double2 ks = kshift[t];
#pragma unroll
    for (int k = 0; k < kZr; ++k) {
        const int c = cg + ng * k;
        if (c < n2) {
            const double d = 0.5 * (kx[a] + ky[b] + kz[c]) + ks.x, w = ks.y;
            const double den = 1.0 / (d * d + w * w);
            const double2 v = acc[k];
            Pz[c * kPencils + j] = double2{(v.x * d - v.y * w) * den, (v.y * d + v.x * w) * den};
        }
    }
    __syncthreads();
    for (int k = 0; k < kZr; ++k) {
        const int zz = cg + ng * k;
        if (zz >= n2) break;
        double sr = 0.0, si = 0.0;
        for (int c = 0; c < n2; ++c) {
            const double u = uz[zz + n2 * c];
            const double2 v = Pz[c * kPencils + j];
            sr += u * v.x;
            si += u * v.y;
        }
        if (xy < P) {
            dr[xy + int64_t(P) * zz] = sr;
            di[xy + int64_t(P) * zz] = si;
        }
    }
}

// ------------------------------------------------------------------ staged step
// pc_step on the plain COCG kernel's z-march (register queue along z, LDS-staged planes, row
// slabs for large planes): q = A p in one sweep over the system, then the pointwise x and r
// updates over the thread's own columns.  One workgroup per slot.
struct LeadSplit {   // the swept vector p, from its real and imaginary columns
    using Buf = double2;
    const double* pr; const double* pi; int P; const int* col;
    __device__ Buf load(int z, int i, bool) const { return load_at(z, unsigned(col[i])); }
    __device__ Buf load_at(int z, unsigned gcol) const {
        const unsigned idx = unsigned(z * P) + gcol;
        return double2{pr[idx], pi[idx]};
    }
    __device__ Buf load_done(int z, unsigned gcol) const { return load_at(z, gcol); }
    __device__ double2 make(const Buf& b) const { return b; }
};
struct CentQ {       // stores q = A p, accumulates p^T q, |p|^2, |q|^2
    using Buf = cocg::Empty;
    double* qr; double* qi; int P; const int* col;
    double acc[4];
    __device__ Buf load(int, int) const { return Buf{}; }
    __device__ void finish(const Buf&, int z, int i, double2 c, double2 q) {
        const unsigned idx = unsigned(z * P + col[i]);
        qr[idx] = q.x;
        qi[idx] = q.y;
        acc[0] += c.x * q.x - c.y * q.y;
        acc[1] += c.x * q.y + c.y * q.x;
        acc[2] += c.x * c.x + c.y * c.y;
        acc[3] += q.x * q.x + q.y * q.y;
    }
};

template <int BSMAX, bool SLAB>
__global__ __attribute__((amdgpu_flat_work_group_size(64, BSMAX)))
void pc_step_wg(PcArgs pa, cocg::Args ca, int it) {
    const int s = blockIdx.x;
    if (!pa.active[s]) return;
    const int sys = pa.order[s];
    cocg::Args a = ca;
    a.omega = pa.omega_v[sys / pa.ns];
    const double eps_n = pa.eps[sys % pa.ns];
    const int tid = threadIdx.x, BS = blockDim.x;
    const int64_t nd = pa.nd;
    extern __shared__ __align__(16) unsigned char smem_pc[];
    double* red = reinterpret_cast<double*>(smem_pc);                  // 16 waves x 8
    double2* planes = reinterpret_cast<double2*>(smem_pc + 16 * 8 * sizeof(double));
    const int nslab = SLAB ? a.nslab : 1;
    cocg::Cols<1> cl;
    cocg::make_cols<1>(a, 0, tid, BS, cl);
    if (!a.periodic) {
        // isolated box: ghost entries read zero (as in the plain kernel)
        const int nent = a.nbuf * (a.rows + 12) * a.rs;
        for (int e = tid; e < nent; e += BS) planes[e] = double2{0.0, 0.0};
        cocg::lds_barrier();
    }
    const double* pr = pa.p + nd * (2 * int64_t(s));
    const double* pi = pr + nd;
    double* qr = pa.q + nd * (2 * int64_t(s));
    double* qi = qr + nd;
    LeadSplit lead{pr, pi, a.P, cl.col};
    CentQ cent{qr, qi, a.P, cl.col, {0.0, 0.0, 0.0, 0.0}};
    double2 Q[13][1];
    for (int sl = 0; sl < nslab; ++sl) {
        if (SLAB) {
            cocg::make_cols<1>(a, sl, tid, BS, cl);
            if (sl > 0) cocg::lds_barrier();
        }
        cocg::march<double, double2, 1, 1, SLAB>(a, cl, planes, eps_n, lead, cent, Q, false);
    }
    if (pa.qonly) return;
    cocg::wg_reduce<4>(cent.acc, red);
    const double s2 = cent.acc[0] * cent.acc[0] + cent.acc[1] * cent.acc[1];
    if (!(s2 > pa.bd_tol * pa.bd_tol * cent.acc[2] * cent.acc[3])) {   // breakdown
        if (tid == 0) {
            pa.iters[sys] = it;
            pa.status[sys] = 2;
            pa.active[s] = 0;
        }
        return;
    }
    const double2 rho = pa.rho[s];
    const double ar = cocg::uniform((rho.x * cent.acc[0] + rho.y * cent.acc[1]) / s2);
    const double ai = cocg::uniform((rho.y * cent.acc[0] - rho.x * cent.acc[1]) / s2);
    double* rr = pa.r + nd * (2 * int64_t(s));
    double* ri = rr + nd;
    double2* xs = pa.x + int64_t(sys) * nd;
    double acc2[1] = {0.0};
    // each thread updates the columns it staged in the sweep (same slab and column mapping),
    // so it reads back only q values it wrote itself
    for (int sl = 0; sl < nslab; ++sl) {
        if (SLAB) cocg::make_cols<1>(a, sl, tid, BS, cl);
        if (!cl.valid[0]) continue;
        for (int z = 0; z < a.n2; ++z) {
            const int64_t i = int64_t(z) * a.P + cl.col[0];
            const double p0r = pr[i], p0i = pi[i], q0r = qr[i], q0i = qi[i];
            double2 xv = xs[i];
            xv.x += ar * p0r - ai * p0i;
            xv.y += ar * p0i + ai * p0r;
            xs[i] = xv;
            const double nr = rr[i] - (ar * q0r - ai * q0i);
            const double ni = ri[i] - (ar * q0i + ai * q0r);
            rr[i] = nr;
            ri[i] = ni;
            acc2[0] += nr * nr + ni * ni;
        }
    }
    cocg::wg_reduce<1>(acc2, red);
    if (tid == 0) {
        pa.iters[sys] = it;
        if (acc2[0] <= pa.tol2 * pa.b2[s]) {
            pa.active[s] = 0;
        } else if (it >= pa.max_iter) {
            pa.status[sys] = 1;
            pa.active[s] = 0;
        }
    }
}

// Launch shape of the staged step: the whole plane with one column per thread when it fits
// 1024 threads, else row slabs of >= 12 rows (as the plain kernel).  Returns false when
// neither fits (the gathered pc_step is used then).
struct StagedShape {
    void (*fn)(PcArgs, cocg::Args, int) = nullptr;
    int bs = 0, nslab = 1, rows = 0, nbuf = 2;
    size_t lds = 0;
};

int pc_lds_row(int n0) { return (n0 + 12 + 7) / 8 * 8; }

bool staged_shape(const Grid& g, StagedShape& sh) {
    const int rs = pc_lds_row(g.n0);
    for (int nslab = 1; nslab <= g.n1 / 12 || nslab == 1; ++nslab) {
        if (g.n1 % nslab != 0) continue;
        const int rows = g.n1 / nslab;
        if (nslab > 1 && rows < 12) break;
        const int bs = (rows * g.n0 + 63) / 64 * 64;
        if (bs > 1024) continue;
        if (nslab > 1 && 12 * g.n0 > bs) continue;
        const int bm = bs <= 512 ? 512 : (bs <= 768 ? 768 : 1024);
        int nbuf = 2;
        size_t lds = 16 * 8 * sizeof(double) + size_t(nbuf) * (rows + 12) * rs * 16;
        if (lds > 150 * 1024) {
            nbuf = 1;
            lds = 16 * 8 * sizeof(double) + size_t(rows + 12) * rs * 16;
        }
        if (lds > 150 * 1024) continue;
        if (nslab == 1)
            sh.fn = bm == 512 ? pc_step_wg<512, false> : bm == 768 ? pc_step_wg<768, false>
                                                                   : pc_step_wg<1024, false>;
        else
            sh.fn = bm == 512 ? pc_step_wg<512, true> : bm == 768 ? pc_step_wg<768, true>
                                                                  : pc_step_wg<1024, true>;
        sh.bs = bs;
        sh.nslab = nslab;
        sh.rows = rows;
        sh.nbuf = nbuf;
        sh.lds = lds;
        return true;
    }
    return false;
}

__global__ __launch_bounds__(PB) void vloc_mean_kernel(int64_t nd, const double* v, double* out) {
    __shared__ double red[PB / 64];
    double acc[1] = {0.0};
    for (int64_t i = threadIdx.x; i < nd; i += PB) acc[0] += v[i];
    pc_reduce<1>(acc, red);
    if (threadIdx.x == 0) *out = acc[0] / double(nd);
}

}  // namespace

hipError_t launch_vloc_mean(int64_t nd, const double* vloc, double* out, hipStream_t s) {
    hipLaunchKernelGGL(vloc_mean_kernel, dim3(1), dim3(PB), 0, s, nd, vloc, out);
    return hipGetLastError();
}

// z = K^{-1} r on the first nsys slots: the fused passes where the grid allows, else the
// Kronecker GEMM passes.
hipError_t apply_precond(const PcocgLaunch& L, int nsys, hipStream_t s) {
    const Grid& g = L.g;
    // RPA_PRECOND_PASSES=gemm forces the GEMM passes, =lds the fused passes wherever their
    // LDS and the pencil pass's z range allow (for measurements)
    static const char* force = std::getenv("RPA_PRECOND_PASSES");
    const int P = g.n0 * g.n1;
    const int64_t nd = g.nd();
    const size_t lxy = size_t(2 * P) * sizeof(double2) +
                       size_t(g.n0 * g.n0 + g.n1 * g.n1) * sizeof(double);
    const size_t lz = size_t(g.n2 * kPencils) * sizeof(double2) + size_t(g.n2 * g.n2) * sizeof(double);
    const bool can = g.n2 <= kZr * (ZB / kPencils) && lxy <= kMaxLds && lz <= kMaxLds &&
                     nsys <= 65535;
    const bool fits = can && g.n0 <= kFusedMaxXY && g.n1 <= kFusedMaxXY && g.n2 <= kFusedMaxZ;
    const bool lds = (force && std::strcmp(force, "lds") == 0) ? can
                   : (force && std::strcmp(force, "gemm") == 0) ? false
                   : fits;
    if (!lds)
        return launch_kron_precond(g, nsys, L.r, L.z, L.tmp, L.Ux, L.Uy, L.Uz, L.kx, L.ky, L.kz,
                                   L.kshift, s);
    hipError_t e;
    if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(pc_xy<false>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, int(lxy))) != hipSuccess)
        return e;
    if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(pc_xy<true>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, int(lxy))) != hipSuccess)
        return e;
    if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(pc_zscale),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, int(lz))) != hipSuccess)
        return e;
    hipLaunchKernelGGL(pc_xy<false>, dim3(unsigned(g.n2), unsigned(nsys)), dim3(XYB), lxy, s, L.r,
                       L.tmp, g.n0, g.n1, nd, L.Ux, L.Uy);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(pc_zscale, dim3(unsigned((P + kPencils - 1) / kPencils), unsigned(nsys)),
                       dim3(ZB), lz, s, L.tmp, g.n0, g.n1, g.n2, nd, L.Uz, L.kx, L.ky, L.kz,
                       L.kshift);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(pc_xy<true>, dim3(unsigned(g.n2), unsigned(nsys)), dim3(XYB), lxy, s, L.tmp,
                       L.z, g.n0, g.n1, nd, L.Ux, L.Uy);
    return hipGetLastError();
}

// Block COCG: the step kernel stores q = A p for the live slots, the block kernels do the
// rest; z aliases r without the preconditioner.  a is the step kernel's argument block.
template <typename Step>
hipError_t run_block(const PcocgLaunch& L, PcArgs& a, dim3 grid, Step& step, int& prefix,
                     hipStream_t s) {
    a.qonly = 1;
    a.boff = L.boff;
    a.split = L.split;
    if (!L.kron) a.z = a.r;
    const dim3 bgrid(unsigned(L.nblk)), bblock(BPB);
    const int sm = L.width <= 2 ? 2 : (L.width <= 4 ? 4 : 8);
    auto update = [&](int it) {
        if (sm == 2) hipLaunchKernelGGL(bc_update<2>, bgrid, bblock, 0, s, a, it);
        else if (sm == 4) hipLaunchKernelGGL(bc_update<4>, bgrid, bblock, 0, s, a, it);
        else hipLaunchKernelGGL(bc_update<8>, bgrid, bblock, 0, s, a, it);
        return hipGetLastError();
    };
    auto dir = [&](int first) {
        if (sm == 2) hipLaunchKernelGGL(bc_dir<2>, bgrid, bblock, 0, s, a, first);
        else if (sm == 4) hipLaunchKernelGGL(bc_dir<4>, bgrid, bblock, 0, s, a, first);
        else hipLaunchKernelGGL(bc_dir<8>, bgrid, bblock, 0, s, a, first);
        return hipGetLastError();
    };
    hipLaunchKernelGGL(pc_start, grid, dim3(PB), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (L.kron && (e = apply_precond(L, prefix, s)) != hipSuccess) return e;
    if ((e = dir(1)) != hipSuccess) return e;
    std::vector<int> act(L.nsys);
    for (int it = 1; it <= L.max_iter; ++it) {
        if ((e = step(it)) != hipSuccess) return e;
        if ((e = update(it)) != hipSuccess) return e;
        if (it % kCheckEvery == 0 || it == L.max_iter) {
            if ((e = hipMemcpyAsync(act.data(), L.active, sizeof(int) * L.nsys,
                                    hipMemcpyDeviceToHost, s)) != hipSuccess)
                return e;
            if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
            prefix = 0;
            for (int t = 0; t < L.nsys; ++t)
                if (act[t]) prefix = t + 1;
            if (prefix == 0) break;
        }
        if (it == L.max_iter) break;
        if (L.kron && (e = apply_precond(L, prefix, s)) != hipSuccess) return e;
        if ((e = dir(0)) != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_pcocg(const PcocgLaunch& L, hipStream_t s) {
    if (L.nsys <= 0) return hipSuccess;
    PcArgs a{};
    a.n0 = L.g.n0;
    a.n1 = L.g.n1;
    a.n2 = L.g.n2;
    a.periodic = L.g.periodic() ? 1 : 0;
    a.nd = L.g.nd();
    double w[7];
    fd_weights(w);
    const double ih2 = 1.0 / (L.g.h * L.g.h);
    a.cw[0] = -0.5 * 3.0 * w[0] * ih2;
    for (int k = 1; k <= 6; ++k) a.cw[k] = -0.5 * w[k] * ih2;
    a.vloc = L.vloc;
    a.eps = L.eps;
    a.omega_v = L.omega_v;
    a.ns = L.ns;
    a.tol2 = L.tol * L.tol;
    a.bd_tol = 1e-14;
    a.max_iter = L.max_iter;
    a.r = L.r;
    a.p = L.p;
    a.z = L.z;
    a.q = L.q;
    a.x = L.x;
    a.rhs = L.rhs;
    a.rho = L.rho;
    a.b2 = L.b2;
    a.active = L.active;
    a.iters = L.iters;
    a.status = L.status;
    a.order = L.order;
    const dim3 grid(unsigned(L.nsys)), block(PB);
    int prefix = L.nsys;   // slots 0 .. prefix-1 hold every system still iterating
    // the staged step (the plain kernel's z-march) where a shape fits, else the gathered one
    StagedShape sh;
    const bool staged = L.g.n2 >= 12 && staged_shape(L.g, sh);
    cocg::Args ca{};
    if (staged) {
        ca.n0 = L.g.n0;
        ca.n1 = L.g.n1;
        ca.n2 = L.g.n2;
        ca.P = L.g.n0 * L.g.n1;
        for (int k = 0; k < 7; ++k) ca.cw[k] = a.cw[k];
        ca.vloc = L.vloc;
        ca.nd = L.g.nd();
        ca.nbuf = sh.nbuf;
        ca.rs = pc_lds_row(L.g.n0);
        ca.periodic = a.periodic;
        ca.nslab = sh.nslab;
        ca.rows = sh.rows;
        hipError_t e0 = hipFuncSetAttribute(reinterpret_cast<const void*>(sh.fn),
                                            hipFuncAttributeMaxDynamicSharedMemorySize,
                                            int(sh.lds));
        if (e0 != hipSuccess) return e0;
    }
    auto step = [&](int it) {
        if (staged)
            hipLaunchKernelGGL(sh.fn, grid, dim3(unsigned(sh.bs)), sh.lds, s, a, ca, it);
        else
            hipLaunchKernelGGL(pc_step, grid, block, 0, s, a, it);
        return hipGetLastError();
    };
    auto precond = [&]() { return apply_precond(L, prefix, s); };
    if (L.width >= 2) return run_block(L, a, grid, step, prefix, s);
    hipLaunchKernelGGL(pc_start, grid, block, 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = precond()) != hipSuccess) return e;
    hipLaunchKernelGGL(pc_rz, grid, dim3(RZB), 0, s, a, 1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    std::vector<int> act(L.nsys);
    for (int it = 1; it <= L.max_iter; ++it) {
        if ((e = step(it)) != hipSuccess) return e;
        if (it % kCheckEvery == 0 || it == L.max_iter) {
            if ((e = hipMemcpyAsync(act.data(), L.active, sizeof(int) * L.nsys,
                                    hipMemcpyDeviceToHost, s)) != hipSuccess)
                return e;
            if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
            prefix = 0;
            for (int t = 0; t < L.nsys; ++t)
                if (act[t]) prefix = t + 1;
            if (prefix == 0) break;
        }
        if (it == L.max_iter) break;
        if ((e = precond()) != hipSuccess) return e;
        hipLaunchKernelGGL(pc_rz, grid, dim3(RZB), 0, s, a, 0);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace rpa
