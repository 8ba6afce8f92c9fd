// FP64 matrix-core (MFMA 16x16x4) GEMMs of the hot path:
//  * occupied projector (Sec. 3, Galerkin removal of occupied components):
//      coeff = dV Psi^T (psi_n .* u_j)          M = N_s, N = N_s*nvec, K = N_d (split-K)
//      r0    = -(psi_n .* u_j - Psi coeff)     M = N_s*nvec, N = N_d, K = N_s
//  * subspace projections (Algorithm 1): C = V^T R, M = R^T R (split-K), V = R L^{-T}
//  * Kronecker transforms of nu^{1/2} (Sec. 3): n x n matrices applied along one axis.
// One workgroup (4 waves) computes a 64 x 64 tile; each wave a 32 x 32 quadrant as 2 x 2
// MFMA blocks.  Operand tiles are staged through LDS by loader functors (bounds-checked),
// so the B operand of the projector (psi_n .* u_j) is formed on the fly and never stored.
// Output tiles are oriented so that the 16 lanes sharing an MFMA row write contiguous
// addresses.
#include <algorithm>
#include <type_traits>

#include "internal.h"

namespace rpa {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 16;
constexpr int NE = BM * BK / 256;   // tile elements loaded per thread and operand

// Loader concept: double operator()(int row, int col, int z) const for A(m, k) or B(k, n),
// plus static constexpr bool k_contig: true if consecutive k are contiguous in memory
// (chooses the thread mapping of the tile load so that loads coalesce).
template <class AL, class BL, class ST>
__global__ __launch_bounds__(256) void gemm_f64(int M, int N, int K, int kchunk, AL al, BL bl,
                                                ST st) {
    __shared__ double As[BK][BM + 1];
    __shared__ double Bs[BK][BN + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN, z = blockIdx.z;
    int kb = 0, ke = K;
    if (kchunk > 0) {
        kb = z * kchunk;
        ke = min(K, kb + kchunk);
    }
    d4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = d4{0, 0, 0, 0};

    // Tile loads for step k0+BK are issued into registers before the MFMAs of step k0, so
    // global (or L2) latency overlaps the matrix-core work.
    double ra[NE], rb[NE];
    // element e of this thread: (row, k) = (tid / BK + (256 / BK) e, tid % BK) when k is
    // contiguous in memory, else (tid % 64, tid / 64 + 4 e)
    auto load_tiles = [&](int k0) {
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            int mm, kk;
            if constexpr (AL::k_contig) {
                kk = tid % BK;
                mm = tid / BK + (256 / BK) * e;
            } else {
                mm = tid & 63;
                kk = (tid >> 6) + 4 * e;
            }
            const int gm = m0 + mm, gk = k0 + kk;
            ra[e] = (gm < M && gk < ke) ? al(gm, gk, z) : 0.0;
        }
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            int nn, kk;
            if constexpr (BL::k_contig) {
                kk = tid % BK;
                nn = tid / BK + (256 / BK) * e;
            } else {
                nn = tid & 63;
                kk = (tid >> 6) + 4 * e;
            }
            const int gn = n0 + nn, gk = k0 + kk;
            rb[e] = (gn < N && gk < ke) ? bl(gk, gn, z) : 0.0;
        }
    };
    if (kb < ke) load_tiles(kb);
    for (int k0 = kb; k0 < ke; k0 += BK) {
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            if constexpr (AL::k_contig) As[tid % BK][tid / BK + (256 / BK) * e] = ra[e];
            else As[(tid >> 6) + 4 * e][tid & 63] = ra[e];
            if constexpr (BL::k_contig) Bs[tid % BK][tid / BK + (256 / BK) * e] = rb[e];
            else Bs[(tid >> 6) + 4 * e][tid & 63] = rb[e];
        }
        __syncthreads();
        if (k0 + BK < ke) load_tiles(k0 + BK);
#pragma unroll
        for (int ks = 0; ks < BK; ks += 4) {
            double af[2], bf[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) af[i] = As[ks + (lane >> 4)][wm * 32 + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < 2; ++j) bf[j] = Bs[ks + (lane >> 4)][wn * 32 + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    // D layout of an FP64 16x16 block: register v of lane l holds row l/16 + 4v, column l%16
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gm = m0 + wm * 32 + i * 16 + (lane >> 4) + 4 * v;
                const int gn = n0 + wn * 32 + j * 16 + (lane & 15);
                if (gm < M && gn < N) st(gm, gn, z, acc[i][j][v]);
            }
}

template <class AL, class BL, class ST>
hipError_t run_gemm(int M, int N, int K, int nz, int kchunk, AL al, BL bl, ST st,
                    hipStream_t s) {
    if (M <= 0 || N <= 0 || nz <= 0) return hipSuccess;
    dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM, nz);
    hipLaunchKernelGGL((gemm_f64<AL, BL, ST>), grid, dim3(256), 0, s, M, N, K, kchunk, al, bl, st);
    return hipGetLastError();
}

// ------------------------------------------------------------------ projector coefficients
struct PsiT {  // A(l, r) = psi[r + nd l]
    static constexpr bool k_contig = true;
    const double* psi; int64_t nd;
    __device__ double operator()(int l, int r, int) const { return psi[r + nd * l]; }
};
struct PsiU {  // B(r, s) = psi[r + nd n] * U[r + nd j], s = n + ns j
    static constexpr bool k_contig = true;
    const double* psi; const double* U; int64_t nd; int ns;
    __device__ double operator()(int r, int s, int) const {
        const int n = s % ns, j = s / ns;
        return psi[r + nd * n] * U[r + nd * j];
    }
};
struct StorePart {  // part[z][l + ns s]
    double* part; int64_t stride; int ldm;
    __device__ void operator()(int m, int n, int z, double v) const {
        part[z * stride + m + int64_t(ldm) * n] = v;
    }
};

__global__ void reduce_parts(const double* part, int nsplit, int64_t n, double scale,
                             double* out) {
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int z = 0; z < nsplit; ++z) s += part[z * n + i];
    out[i] = scale * s;
}

// ------------------------------------------------------------------ projected RHS
struct CoeffT {  // A(s, l) = coeff[l + ns s]
    static constexpr bool k_contig = true;
    const double* coeff; int ns;
    __device__ double operator()(int s, int l, int) const { return coeff[l + ns * s]; }
};
struct PsiKN {  // B(l, r) = psi[r + nd l]
    static constexpr bool k_contig = false;
    const double* psi; int64_t nd;
    __device__ double operator()(int l, int r, int) const { return psi[r + nd * l]; }
};
template <typename T>
struct StoreRhs {  // r0[s][r] = -(psi_n u_j - acc), complex with zero imaginary part
    const double* psi; const double* U; int64_t nd; int ns; T* r0; double* r64;
    __device__ void operator()(int s, int r, int, double acc) const {
        const int n = s % ns, j = s / ns;
        const double b = psi[r + nd * n] * U[r + nd * j] - acc;
        using T2 = typename std::conditional<std::is_same<T, float>::value, float2, double2>::type;
        reinterpret_cast<T2*>(r0)[int64_t(s) * nd + r] = T2{T(-b), T(0)};
        if (r64)   // the same right-hand side as complex float64
            reinterpret_cast<double2*>(r64)[int64_t(s) * nd + r] = double2{-b, 0.0};
    }
};

// ------------------------------------------------------------------ Gram and rotation
struct ColT {  // A(i, k) = A[k + nd i]   (operand transposed)
    static constexpr bool k_contig = true;
    const double* A; int64_t nd;
    __device__ double operator()(int i, int k, int) const { return A[k + nd * i]; }
};
struct ColN {  // B(k, j) = B[k + nd j]
    static constexpr bool k_contig = true;
    const double* B; int64_t nd;
    __device__ double operator()(int k, int j, int) const { return B[k + nd * j]; }
};
struct SmallT {  // A(nn, k) = T[k + m nn]
    static constexpr bool k_contig = true;
    const double* T; int m;
    __device__ double operator()(int nn, int k, int) const { return T[k + m * nn]; }
};
struct TallKN {  // B(k, r) = A[r + nd k]
    static constexpr bool k_contig = false;
    const double* A; int64_t nd;
    __device__ double operator()(int k, int r, int) const { return A[r + nd * k]; }
};
struct StoreColMajor {  // Y[n + nd m]  (m = column index, n = row index of Y)
    double* Y; int64_t nd;
    __device__ void operator()(int m, int n, int, double v) const { Y[n + nd * m] = v; }
};

// ------------------------------------------------------------------ Kronecker transforms
// Axis transforms on X (n0 x n1 x n2 x nvec, x fastest).  Forward: c_a = sum_t U[t + n a] f_t;
// inverse: f_t = sum_a U[t + n a] c_a.
struct AxisX {  // A(rest, t) = X[t + n0 rest]
    static constexpr bool k_contig = true;
    const double* X; int n0;
    __device__ double operator()(int rest, int t, int) const { return X[t + int64_t(n0) * rest]; }
};
struct BasisB {  // forward: B(t, a) = U[t + n a]; inverse: B(a, t) = U[t + n a]
    static constexpr bool k_contig = true;
    const double* U; int n; bool inverse;
    __device__ double operator()(int k, int c, int) const {
        return inverse ? U[c + n * k] : U[k + n * c];
    }
};
struct StoreX {  // Y[a + n0 rest]
    double* Y; int n0;
    __device__ void operator()(int rest, int a, int, double v) const { Y[a + int64_t(n0) * rest] = v; }
};
struct BasisA {  // forward: A(b, t) = U[t + n b]; inverse: A(t, b) = U[t + n b]
    static constexpr bool k_contig = true;
    const double* U; int n; bool inverse;
    __device__ double operator()(int mrow, int k, int) const {
        return inverse ? U[mrow + n * k] : U[k + n * mrow];
    }
};
struct AxisY {  // B(t, x) = X[x + n0 (t + n1 zslab)], z = slab index (z-plane and vector)
    static constexpr bool k_contig = false;
    const double* X; int n0, n1;
    __device__ double operator()(int t, int x, int zs) const {
        return X[x + int64_t(n0) * (t + int64_t(n1) * zs)];
    }
};
struct StoreY {  // Y[x + n0 (b + n1 zs)]
    double* Y; int n0, n1;
    __device__ void operator()(int b, int x, int zs, double v) const {
        Y[x + int64_t(n0) * (b + int64_t(n1) * zs)] = v;
    }
};
struct AxisZ {  // B(t, xy) = X[xy + P (t + n2 j)], z = vector j
    static constexpr bool k_contig = false;
    const double* X; int P, n2;
    __device__ double operator()(int t, int xy, int j) const {
        return X[xy + int64_t(P) * (t + int64_t(n2) * j)];
    }
};
struct StoreZ {  // Y[xy + P (c + n2 j)]
    double* Y; int P, n2;
    __device__ void operator()(int c, int xy, int j, double v) const {
        Y[xy + int64_t(P) * (c + int64_t(n2) * j)] = v;
    }
};

// s^power = (4 pi / (kx + ky + kz))^{power/2} per mode; zero_mode: the all-zero-index mode (the
// constant of a periodic grid) is the null space and gets 0.
__global__ void kron_scale(double* X, int n0, int n1, int n2, int64_t total, const double* kx,
                           const double* ky, const double* kz, int power, int zero_mode) {
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i >= total) return;
    const int64_t nd = int64_t(n0) * n1 * n2;
    const int64_t p = i % nd;
    const int x = int(p % n0), y = int((p / n0) % n1), z = int(p / (int64_t(n0) * n1));
    double s = 0.0;
    if (!zero_mode || x != 0 || y != 0 || z != 0) {
        const double K = kx[x] + ky[y] + kz[z];
        s = (power == 2) ? 4.0 * M_PI / K : sqrt(4.0 * M_PI / K);
    }
    X[i] *= s;
}

// Preconditioner scale on the mode grid: columns 2t and 2t+1 are the real and imaginary
// parts of system t; each mode is divided by 1/2 (kx + ky + kz) + sigma_t - i omega_t, with
// kshift[t] = (sigma_t, omega_t).
__global__ void precond_scale(double* X, int n0, int n1, int n2, int64_t npair,
                              const double* kx, const double* ky, const double* kz,
                              const double2* kshift) {
    const int64_t nd = int64_t(n0) * n1 * n2;
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i >= nd * npair) return;
    const int64_t p = i % nd, t = i / nd;
    const int x = int(p % n0), y = int((p / n0) % n1), z = int(p / (int64_t(n0) * n1));
    const double2 ks = kshift[t];
    const double d = 0.5 * (kx[x] + ky[y] + kz[z]) + ks.x, w = ks.y;
    const double den = 1.0 / (d * d + w * w);
    double* re = X + p + nd * (2 * t);
    double* im = re + nd;
    const double a = *re, b = *im;
    *re = (a * d - b * w) * den;
    *im = (b * d + a * w) * den;
}

struct W7 {
    double w[7];
};

__global__ void eigbasis_kernel(int n, double h, W7 wt, double* U, double* kappa) {
    const double* w = wt.w;
    // Real Fourier basis of the periodic circulant -D2: column 0 constant, then cos/sin
    // pairs, and for even n the alternating mode.  kappa(theta) = h^-2 (-w0 - 2 sum w_p cos p theta).
    const int a = blockIdx.x;      // mode (column)
    const int t = threadIdx.x;     // grid point (row)
    int k;
    bool is_sin = false;
    if (a == 0) {
        k = 0;
    } else {
        k = (a + 1) / 2;
        is_sin = (a % 2 == 0);
        if (n % 2 == 0 && a == n - 1) { k = n / 2; is_sin = false; }
    }
    const double th = 2.0 * M_PI * double(k) / double(n);
    if (t < n) {
        double v;
        if (k == 0) v = 1.0 / sqrt(double(n));
        else if (n % 2 == 0 && k == n / 2) v = ((t & 1) ? -1.0 : 1.0) / sqrt(double(n));
        else v = sqrt(2.0 / double(n)) * (is_sin ? sin(th * t) : cos(th * t));
        U[t + int64_t(n) * a] = v;
    }
    if (t == 0) {
        double s = -w[0];
        for (int p = 1; p <= 6; ++p) s -= 2.0 * w[p] * cos(p * th);
        kappa[a] = (k == 0) ? 0.0 : s / (h * h);
    }
}

}  // namespace

// Projector coefficients when all N_s orbitals fit one 64-row tile (N_s <= 64): the B
// operand psi_n .* u_j reuses the Psi tile already staged for A.  Per K step the workgroup
// loads the 64 x 16 Psi tile and the few U columns its 64 output columns touch (columns
// s = n + ns j of one tile span at most 64/ns + 1 values of j), and each B fragment is formed
// in the MFMA loop as As[k][n] * Us[k][j - j_first].  Half the global loads of the general
// loader, no extra barrier.  Same tile, wave and output layout as gemm_f64.
__global__ __launch_bounds__(256) void gemm_coeff_f64(int ns, int S, int K, int kchunk,
                                                      const double* __restrict__ psi,
                                                      const double* __restrict__ U, int64_t nd,
                                                      double* part, int64_t pstride) {
    __shared__ double As[BK][BM + 1];
    __shared__ double Us[BK][BN + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int n0 = blockIdx.x * BN, z = blockIdx.z;
    const int kb = z * kchunk, ke = min(K, kb + kchunk);
    const int jfirst = n0 / ns;
    const int nj = min(BN, (min(S, n0 + BN) - 1) / ns - jfirst + 1);   // distinct j in the tile
    d4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = d4{0, 0, 0, 0};
    // this lane's B columns: orbital row in As and U column in Us (fixed over k)
    int brow[2], bcol[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int gn = min(S - 1, n0 + wn * 32 + j * 16 + (lane & 15));
        brow[j] = gn % ns;
        bcol[j] = gn / ns - jfirst;
    }
    // tile element e of this thread: k = tid % BK, row = tid / BK + 16 e (k contiguous)
    double ra[NE], ru[NE];
    auto load_tiles = [&](int k0) {
        const int kk = tid % BK, gk = k0 + kk;
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            const int mm = tid / BK + (256 / BK) * e;
            ra[e] = (mm < ns && gk < ke) ? psi[gk + nd * mm] : 0.0;
            ru[e] = (mm < nj && gk < ke) ? U[gk + nd * (jfirst + mm)] : 0.0;
        }
    };
    if (kb < ke) load_tiles(kb);
    for (int k0 = kb; k0 < ke; k0 += BK) {
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            As[tid % BK][tid / BK + (256 / BK) * e] = ra[e];
            Us[tid % BK][tid / BK + (256 / BK) * e] = ru[e];
        }
        __syncthreads();
        if (k0 + BK < ke) load_tiles(k0 + BK);
#pragma unroll
        for (int ks = 0; ks < BK; ks += 4) {
            const int kr = ks + (lane >> 4);
            double af[2], bf[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) af[i] = As[kr][wm * 32 + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < 2; ++j) bf[j] = As[kr][brow[j]] * Us[kr][bcol[j]];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gm = wm * 32 + i * 16 + (lane >> 4) + 4 * v;
                const int gn = n0 + wn * 32 + j * 16 + (lane & 15);
                if (gm < ns && gn < S) part[z * pstride + gm + int64_t(ns) * gn] = acc[i][j][v];
            }
}

hipError_t launch_proj_coeff(int64_t nd, int ns, int nvec, double dV, const double* psi,
                             const double* U, double* part, int nsplit, double* coeff,
                             hipStream_t s) {
    const int S = ns * nvec;
    const int kchunk = int((nd + nsplit - 1) / nsplit + BK - 1) / BK * BK;
    const int nz = int((nd + kchunk - 1) / kchunk);
    hipError_t e;
    if (ns <= BM && S > 0) {
        hipLaunchKernelGGL(gemm_coeff_f64, dim3(unsigned((S + BN - 1) / BN), 1, unsigned(nz)),
                           dim3(256), 0, s, ns, S, int(nd), kchunk, psi, U, nd, part,
                           int64_t(ns) * S);
        e = hipGetLastError();
    } else {
        e = run_gemm(ns, S, int(nd), nz, kchunk, PsiT{psi, nd}, PsiU{psi, U, nd, ns},
                     StorePart{part, int64_t(ns) * S, ns}, s);
    }
    if (e != hipSuccess) return e;
    const int64_t n = int64_t(ns) * S;
    hipLaunchKernelGGL(reduce_parts, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, part, nz,
                       n, dV, coeff);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_proj_rhs(int64_t nd, int ns, int nvec, const double* psi, const double* U,
                           const double* coeff, T* r0, double* r64, hipStream_t s) {
    const int S = ns * nvec;
    return run_gemm(S, int(nd), ns, 1, 0, CoeffT{coeff, ns}, PsiKN{psi, nd},
                    StoreRhs<T>{psi, U, nd, ns, r0, r64}, s);
}
template hipError_t launch_proj_rhs<double>(int64_t, int, int, const double*, const double*,
                                            const double*, double*, double*, hipStream_t);
template hipError_t launch_proj_rhs<float>(int64_t, int, int, const double*, const double*,
                                           const double*, float*, double*, hipStream_t);

hipError_t launch_gram(int64_t nd, int m, const double* A, const double* B, double* part,
                       int nsplit, double* G, hipStream_t s) {
    const int kchunk = int((nd + nsplit - 1) / nsplit + BK - 1) / BK * BK;
    const int nz = int((nd + kchunk - 1) / kchunk);
    hipError_t e = run_gemm(m, m, int(nd), nz, kchunk, ColT{A, nd}, ColN{B, nd},
                            StorePart{part, int64_t(m) * m, m}, s);
    if (e != hipSuccess) return e;
    const int64_t n = int64_t(m) * m;
    hipLaunchKernelGGL(reduce_parts, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, part, nz,
                       n, 1.0, G);
    return hipGetLastError();
}

hipError_t launch_gemm_tall_small(int64_t nd, int m, const double* A, const double* T,
                                  double* Y, hipStream_t s) {
    // Y^T = T^T A^T: rows of the product are columns of Y, so lanes run along the grid.
    return run_gemm(m, int(nd), m, 1, 0, SmallT{T, m}, TallKN{A, nd}, StoreColMajor{Y, nd}, s);
}

hipError_t launch_eigbasis_1d(int n, double h, double* U, double* kappa, hipStream_t s) {
    W7 wt;
    fd_weights(wt.w);
    hipLaunchKernelGGL(eigbasis_kernel, dim3(n), dim3((n + 63) / 64 * 64), 0, s, n, h, wt, U,
                       kappa);
    return hipGetLastError();
}

// A = -D2 of an isolated box: A[i + n j] = -w_|i-j| / h^2 for |i - j| <= 6 (reaches beyond the
// walls dropped)
__global__ void box_matrix_kernel(int n, double h, W7 wt, double* A) {
    const int j = blockIdx.x, i = threadIdx.x;
    if (i >= n) return;
    const int d = i > j ? i - j : j - i;
    A[i + int64_t(n) * j] = (d <= 6) ? -wt.w[d] / (h * h) : 0.0;
}

hipError_t launch_eigbasis_1d_box(int n, double h, double* U, double* kappa, double* work,
                                  hipStream_t s) {
    W7 wt;
    fd_weights(wt.w);
    double* A = work;
    hipLaunchKernelGGL(box_matrix_kernel, dim3(n), dim3((n + 63) / 64 * 64), 0, s, n, h, wt, A);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_syevj(n, A, work + int64_t(n) * n, kappa, U, s);
}

static hipError_t kron_chunk(const Grid& g, int power, int nvec, const double* in, double* out,
                             double* tmp, const double* Ux, const double* Uy, const double* Uz,
                             const double* kx, const double* ky, const double* kz,
                             hipStream_t s, const double2* kshift = nullptr) {
    const int n0 = g.n0, n1 = g.n1, n2 = g.n2, P = n0 * n1;
    const int rows_x = n1 * n2 * nvec;
    hipError_t e;
    // forward x: tmp(rest, a) = sum_t in(t, rest) Ux[t + n0 a]
    e = run_gemm(rows_x, n0, n0, 1, 0, AxisX{in, n0}, BasisB{Ux, n0, false}, StoreX{tmp, n0}, s);
    if (e != hipSuccess) return e;
    // forward y: out(b, x) per slab = sum_t Uy[t + n1 b] tmp(x, t)
    e = run_gemm(n1, n0, n1, n2 * nvec, 0, BasisA{Uy, n1, false}, AxisY{tmp, n0, n1},
                 StoreY{out, n0, n1}, s);
    if (e != hipSuccess) return e;
    // forward z: tmp(c, xy) per vector = sum_t Uz[t + n2 c] out(xy, t)
    e = run_gemm(n2, P, n2, nvec, 0, BasisA{Uz, n2, false}, AxisZ{out, P, n2}, StoreZ{tmp, P, n2},
                 s);
    if (e != hipSuccess) return e;
    const int64_t total = g.nd() * nvec;
    if (kshift)
        hipLaunchKernelGGL(precond_scale, dim3(unsigned((total + 255) / 256)), dim3(256), 0, s,
                           tmp, n0, n1, n2, int64_t(nvec / 2), kx, ky, kz, kshift);
    else
        hipLaunchKernelGGL(kron_scale, dim3(unsigned((total + 255) / 256)), dim3(256), 0, s, tmp,
                           n0, n1, n2, total, kx, ky, kz, power, g.periodic() ? 1 : 0);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    // inverse z, y, x
    e = run_gemm(n2, P, n2, nvec, 0, BasisA{Uz, n2, true}, AxisZ{tmp, P, n2}, StoreZ{out, P, n2},
                 s);
    if (e != hipSuccess) return e;
    e = run_gemm(n1, n0, n1, n2 * nvec, 0, BasisA{Uy, n1, true}, AxisY{out, n0, n1},
                 StoreY{tmp, n0, n1}, s);
    if (e != hipSuccess) return e;
    return run_gemm(rows_x, n0, n0, 1, 0, AxisX{tmp, n0}, BasisB{Ux, n0, true}, StoreX{out, n0},
                    s);
}

hipError_t launch_kron_apply(const Grid& g, int power, int nvec, const double* in, double* out,
                             double* tmp, const double* Ux, const double* Uy, const double* Uz,
                             const double* kx, const double* ky, const double* kz,
                             hipStream_t s) {
    // keep every launch within the grid limits: gridDim.z = n2 * chunk (y pass) and
    // gridDim.y = n1 * n2 * chunk / 64 (x pass) must stay below 65536
    const int64_t lim_y = 65535 / g.n2;
    const int64_t lim_x = (int64_t(65535) * BM) / (int64_t(g.n1) * g.n2);
    const int chunk = int(std::max<int64_t>(1, std::min<int64_t>({int64_t(nvec), lim_y, lim_x})));
    const int64_t nd = g.nd();
    for (int j0 = 0; j0 < nvec; j0 += chunk) {
        const int nv = std::min(chunk, nvec - j0);
        hipError_t e = kron_chunk(g, power, nv, in + nd * j0, out + nd * j0, tmp + nd * j0, Ux, Uy,
                                  Uz, kx, ky, kz, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_kron_precond(const Grid& g, int nsys, const double* in, double* out,
                               double* tmp, const double* Ux, const double* Uy, const double* Uz,
                               const double* kx, const double* ky, const double* kz,
                               const double2* kshift, hipStream_t s) {
    // as launch_kron_apply, on 2 nsys columns kept in (real, imaginary) pairs per chunk
    const int64_t lim_y = 65535 / g.n2;
    const int64_t lim_x = (int64_t(65535) * BM) / (int64_t(g.n1) * g.n2);
    const int64_t ncol = 2 * int64_t(nsys);
    int chunk = int(std::max<int64_t>(2, std::min<int64_t>({ncol, lim_y, lim_x})));
    chunk -= chunk % 2;
    const int64_t nd = g.nd();
    for (int64_t j0 = 0; j0 < ncol; j0 += chunk) {
        const int nv = int(std::min<int64_t>(chunk, ncol - j0));
        hipError_t e = kron_chunk(g, 0, nv, in + nd * j0, out + nd * j0, tmp + nd * j0, Ux, Uy,
                                  Uz, kx, ky, kz, s, kshift + j0 / 2);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace rpa
