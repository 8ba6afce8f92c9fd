// Small dense FP64 kernels of the subspace step (Algorithm 1) and the pointwise epilogues.
//  * Cholesky of the N_r x N_r overlap M = R^T R and T = L^{-T}, so V = R T (orthonormalisation)
//  * E_{c,m} = W/(2 pi) sum_k g(mu_k) through sum_k g(mu_k) = ln det(I - C) + tr C, with
//    I - C symmetric positive definite because C <= 0 (Eq. 10)
//  * cyclic Jacobi eigensolver for the Ritz values and vectors of C (Rayleigh-Ritz)
//  * Delta rho = 4 sum_n psi_n Re(x_n) (Eq. 8) and the gradient accumulation
// Each small-matrix kernel runs as one workgroup of 1024 threads: up to N_r = 90 the
// matrices are factorised in LDS, beyond that in place in global memory (L2-resident); N_r is
// at most a few hundred, so these are latency-bound and a small share of a subspace
// iteration.
#include "internal.h"

namespace rpa {
namespace {

constexpr int SB = 1024;

__device__ double block_sum(double v, double* red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[w];
    __syncthreads();
    return s;
}

// Lower Cholesky factor of the m x m column-major matrix A into L (upper part zeroed),
// left-looking, one column per step.  Returns through info: 0 or (failing column + 1).
__device__ void chol_block(int m, const double* A, double* L, int* info, double* rowj,
                           int* sflag) {
    const int tid = threadIdx.x, bs = blockDim.x;
    for (int i = tid; i < m * m; i += bs) {
        const int r = i % m, c = i / m;
        L[i] = (r >= c) ? A[i] : 0.0;
    }
    if (tid == 0) *sflag = 0;
    __syncthreads();
    for (int j = 0; j < m; ++j) {
        for (int k = tid; k < j; k += bs) rowj[k] = L[j + int64_t(m) * k];
        __syncthreads();
        for (int i = j + tid; i < m; i += bs) {
            double s = L[i + int64_t(m) * j];
            for (int k = 0; k < j; ++k) s -= L[i + int64_t(m) * k] * rowj[k];
            L[i + int64_t(m) * j] = s;
        }
        __syncthreads();
        if (tid == 0) {
            const double d = L[j + int64_t(m) * j];
            if (!(d > 0.0) && *sflag == 0) *sflag = j + 1;
            L[j + int64_t(m) * j] = (d > 0.0) ? sqrt(d) : 1.0;
        }
        __syncthreads();
        const double piv = L[j + int64_t(m) * j];
        for (int i = j + 1 + tid; i < m; i += bs) L[i + int64_t(m) * j] /= piv;
        __syncthreads();
    }
    if (tid == 0) *info = *sflag;
    __syncthreads();
}

__global__ __launch_bounds__(SB) void chol_inv_kernel(int m, const double* M, double* L,
                                                      double* T, int* info) {
    extern __shared__ double sh[];
    __shared__ int sflag;
    chol_block(m, M, L, info, sh, &sflag);
    // T = (L^{-1})^T: thread c solves L x = e_c by forward substitution, x_i = T[c + m i]
    for (int c = threadIdx.x; c < m; c += blockDim.x) {
        for (int i = 0; i < c; ++i) T[c + int64_t(m) * i] = 0.0;
        for (int i = c; i < m; ++i) {
            double s = (i == c) ? 1.0 : 0.0;
            for (int k = c; k < i; ++k) s -= L[i + int64_t(m) * k] * T[c + int64_t(m) * k];
            T[c + int64_t(m) * i] = s / L[i + int64_t(m) * i];
        }
    }
}

__global__ __launch_bounds__(SB) void energy_kernel(int m, const double* C, double scale,
                                                    double* work, double* out, int* info) {
    extern __shared__ double sh[];
    __shared__ int sflag;
    __shared__ double red[SB / 64];
    double* B = work;                 // I - C
    double* L = work + int64_t(m) * m;
    for (int i = threadIdx.x; i < m * m; i += blockDim.x) {
        const int r = i % m, c = i / m;
        B[i] = (r == c ? 1.0 : 0.0) - C[i];
    }
    __syncthreads();
    chol_block(m, B, L, info, sh, &sflag);
    double v = 0.0;
    for (int i = threadIdx.x; i < m; i += blockDim.x)
        v += 2.0 * log(L[i + int64_t(m) * i]) + C[i + int64_t(m) * i];
    const double s = block_sum(v, red);
    if (threadIdx.x == 0) out[0] = scale * s;
}

// Small N_r (the whole matrix in LDS): right-looking Cholesky in place on the lower
// triangle of the m x m column-major LDS matrix A.  sflag = failing column + 1, or 0.
__device__ void chol_lds(int m, double* A, int* sflag) {
    const int tid = threadIdx.x, bs = blockDim.x;
    for (int j = 0; j < m; ++j) {
        if (tid == 0) {
            const double d = A[j + m * j];
            if (!(d > 0.0) && *sflag == 0) *sflag = j + 1;
            A[j + m * j] = (d > 0.0) ? sqrt(d) : 1.0;
        }
        __syncthreads();
        const double piv = A[j + m * j];
        for (int i = j + 1 + tid; i < m; i += bs) A[i + m * j] /= piv;
        __syncthreads();
        // trailing update of the lower triangle, columns k and rows i in (j, m), i >= k
        const int n = m - j - 1;
        for (int e = tid; e < n * n; e += bs) {
            const int i = j + 1 + e % n, k = j + 1 + e / n;
            if (i >= k) A[i + m * k] -= A[i + m * j] * A[k + m * j];
        }
        __syncthreads();
    }
}

// chol_inv for small m: M -> L (LDS), X = L^{-1} column by column (thread per column,
// forward substitution from LDS), T = X^T.
__global__ __launch_bounds__(SB) void chol_inv_lds_kernel(int m, const double* M, double* L,
                                                          double* T, int* info) {
    extern __shared__ double sh[];
    __shared__ int sflag;
    double* A = sh;
    double* X = sh + m * m;
    const int tid = threadIdx.x, bs = blockDim.x;
    for (int i = tid; i < m * m; i += bs) {
        const int r = i % m, c = i / m;
        A[i] = (r >= c) ? M[i] : 0.0;
    }
    if (tid == 0) sflag = 0;
    __syncthreads();
    chol_lds(m, A, &sflag);
    for (int c = tid; c < m; c += bs) {
        X[c + m * c] = 1.0 / A[c + m * c];
        for (int i = c + 1; i < m; ++i) {
            double acc = 0.0;
            for (int k = c; k < i; ++k) acc += A[i + m * k] * X[k + m * c];
            X[i + m * c] = -acc / A[i + m * i];
        }
    }
    __syncthreads();
    for (int e = tid; e < m * m; e += bs) {
        const int r = e % m, c = e / m;
        T[e] = (c >= r) ? X[c + m * r] : 0.0;
        L[e] = A[e];
    }
    if (tid == 0) *info = sflag;
}

// energy for small m: Cholesky of I - C in LDS, then ln det + tr.
__global__ __launch_bounds__(SB) void energy_lds_kernel(int m, const double* C, double scale,
                                                        double* out, int* info) {
    extern __shared__ double sh[];
    __shared__ int sflag;
    __shared__ double red[SB / 64];
    double* A = sh;
    const int tid = threadIdx.x, bs = blockDim.x;
    for (int i = tid; i < m * m; i += bs) {
        const int r = i % m, c = i / m;
        A[i] = (r >= c) ? ((r == c ? 1.0 : 0.0) - C[i]) : 0.0;
    }
    if (tid == 0) sflag = 0;
    __syncthreads();
    chol_lds(m, A, &sflag);
    double v = 0.0;
    for (int i = tid; i < m; i += bs) v += 2.0 * log(A[i + m * i]) + C[i + int64_t(m) * i];
    const double sum = block_sum(v, red);
    if (tid == 0) {
        out[0] = scale * sum;
        *info = sflag;
    }
}

// LDS budget of the small-matrix path (both chol_inv buffers)
constexpr int kSmallLdsBytes = 128 * 1024;

__global__ void symmetrize_kernel(int m, double* C) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m * m) return;
    const int r = i % m, c = i / m;
    if (r < c) {
        const double a = C[r + int64_t(m) * c], b = C[c + int64_t(m) * r];
        const double s = 0.5 * (a + b);
        C[r + int64_t(m) * c] = s;
        C[c + int64_t(m) * r] = s;
    }
}

// Cyclic Jacobi with the round-robin ordering: each step rotates m/2 disjoint pairs at once.
__global__ __launch_bounds__(SB) void syevj_kernel(int m, const double* Ain, double* work,
                                                   double* w, double* Yout) {
    extern __shared__ double sh[];  // cs[2 * mm/2] then diag copy
    __shared__ double red[SB / 64];
    const int tid = threadIdx.x, bs = blockDim.x;
    const int mm = m + (m & 1);
    const int np = mm / 2;
    double* A = work;
    double* Y = work + int64_t(m) * m;
    double* cs = sh;                 // 2*np
    int* pp = reinterpret_cast<int*>(sh + 2 * np);  // 2*np ints
    for (int i = tid; i < m * m; i += bs) {
        A[i] = 0.5 * (Ain[i] + Ain[(i / m) + int64_t(m) * (i % m)]);
        Y[i] = (i % m == i / m) ? 1.0 : 0.0;
    }
    __syncthreads();
    double fro = 0.0;
    for (int i = tid; i < m * m; i += bs) fro += A[i] * A[i];
    fro = block_sum(fro, red);
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0;
        for (int i = tid; i < m * m; i += bs)
            if (i % m != i / m) off += A[i] * A[i];
        off = block_sum(off, red);
        if (!(off > 1e-30 * fro) || fro == 0.0) break;
        for (int t = 0; t < mm - 1; ++t) {
            for (int k = tid; k < np; k += bs) {
                const int a0 = (k == 0) ? 0 : ((k - 1 + t) % (mm - 1)) + 1;
                const int k2 = mm - 1 - k;
                const int b0 = ((k2 - 1 + t) % (mm - 1)) + 1;
                int p = min(a0, b0), q = max(a0, b0);
                double c = 1.0, s = 0.0;
                if (q < m) {
                    const double apq = A[p + int64_t(m) * q];
                    if (apq != 0.0) {
                        const double app = A[p + int64_t(m) * p], aqq = A[q + int64_t(m) * q];
                        const double tau = (aqq - app) / (2.0 * apq);
                        const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + tt * tt);
                        s = tt * c;
                    }
                } else {
                    p = q = -1;
                }
                cs[2 * k] = c;
                cs[2 * k + 1] = s;
                pp[2 * k] = p;
                pp[2 * k + 1] = q;
            }
            __syncthreads();
            // rows: A <- J^T A
            for (int it = tid; it < np * m; it += bs) {
                const int k = it / m, col = it % m;
                const int p = pp[2 * k], q = pp[2 * k + 1];
                if (p < 0) continue;
                const double c = cs[2 * k], s = cs[2 * k + 1];
                const double ap = A[p + int64_t(m) * col], aq = A[q + int64_t(m) * col];
                A[p + int64_t(m) * col] = c * ap - s * aq;
                A[q + int64_t(m) * col] = s * ap + c * aq;
            }
            __syncthreads();
            // columns: A <- A J, Y <- Y J
            for (int it = tid; it < np * m; it += bs) {
                const int k = it / m, row = it % m;
                const int p = pp[2 * k], q = pp[2 * k + 1];
                if (p < 0) continue;
                const double c = cs[2 * k], s = cs[2 * k + 1];
                double ap = A[row + int64_t(m) * p], aq = A[row + int64_t(m) * q];
                A[row + int64_t(m) * p] = c * ap - s * aq;
                A[row + int64_t(m) * q] = s * ap + c * aq;
                ap = Y[row + int64_t(m) * p];
                aq = Y[row + int64_t(m) * q];
                Y[row + int64_t(m) * p] = c * ap - s * aq;
                Y[row + int64_t(m) * q] = s * ap + c * aq;
            }
            __syncthreads();
        }
    }
    // sort ascending (stable by index)
    for (int i = tid; i < m; i += bs) {
        const double di = A[i + int64_t(m) * i];
        int rank = 0;
        for (int j = 0; j < m; ++j) {
            const double dj = A[j + int64_t(m) * j];
            rank += (dj < di) || (dj == di && j < i);
        }
        w[rank] = di;
        if (Yout)
            for (int r = 0; r < m; ++r) Yout[r + int64_t(m) * rank] = Y[r + int64_t(m) * i];
    }
}

template <int STRIDE>
__global__ void drho_kernel(int64_t nd, int ns, const double* psi, const double* x, double* out) {
    const int64_t r = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    const int j = blockIdx.y;
    if (r >= nd) return;
    double s = 0.0;
    for (int n = 0; n < ns; ++n)
        s += psi[r + nd * n] * x[STRIDE * ((int64_t(n) + int64_t(ns) * j) * nd + r)];
    out[r + nd * j] = 4.0 * s;
}

// d[l, s] = coeff[l, s] / (eps_l - eps_n - i omega), s = n + ns k
__global__ void grad_d_kernel(int ns, int S, const double* eps, double omega, const double* coeff,
                              double2* d) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ns * S) return;
    const int l = i % ns, s = i / ns, n = s % ns;
    const double a = eps[l] - eps[n], b = -omega;   // denominator a + i b
    const double den = a * a + b * b;
    const double c = coeff[i];
    d[i] = double2{c * a / den, -c * b / den};
}

template <typename T2, int NSMAX>
__global__ void grad_kernel(int64_t nd, int ns, int nvec, const double* psi, const double2* d,
                            const double* coefk, const T2* x, double* grad) {
    const int64_t r = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (r >= nd) return;
    double pr[NSMAX];
#pragma unroll
    for (int l = 0; l < NSMAX; ++l) pr[l] = (l < ns) ? psi[r + nd * l] : 0.0;
    double acc = 0.0;
    for (int k = 0; k < nvec; ++k) {
        double ak = 0.0;
        for (int n = 0; n < ns; ++n) {
            const int s = n + ns * k;
            double ore = 0.0, oim = 0.0;
#pragma unroll
            for (int l = 0; l < NSMAX; ++l) {
                if (l < ns) {
                    const double2 dl = d[l + int64_t(ns) * s];
                    ore -= pr[l] * dl.x;
                    oim -= pr[l] * dl.y;
                }
            }
            const T2 xv = x[int64_t(s) * nd + r];
            const double xr = double(xv.x), xi = double(xv.y);
            // Re[(x + o) x]
            ak += (xr + ore) * xr - (xi + oim) * xi;
        }
        acc += coefk[k] * 4.0 * ak;
    }
    grad[r] += acc;
}

__global__ void scale_kernel(int64_t n, double a, double* x) {
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i < n) x[i] *= a;
}
__global__ void fill_kernel(int64_t n, double v, double* x) {
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i < n) x[i] = v;
}
__global__ void copy_kernel(int64_t n, const double* src, double* dst) {
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// ------------------------------------------------------------------ Gauss spectral quadrature
// E = scale * sum_r sum_t Q_r(1,t)^2 g(lambda_t): for each standard basis vector e_r, n_o
// Lanczos steps on C give the tridiagonal J_r, whose eigenvalues (nodes) and squared first
// eigenvector components (weights) form the Gauss rule for e_r^T g(C) e_r (Sec. 3,
// Algorithm 1, SQ method).  One workgroup per r; the m x m matrix C is read once per step
// (coalesced along columns); Lanczos stops early when beta <= 1e-14 max|C| (exhausted Krylov
// space).  The small tridiagonal eigenproblem is solved by cyclic Jacobi on one wave.

__global__ __launch_bounds__(256) void absmax_kernel(int64_t n, const double* a, double* out) {
    __shared__ double red[4];
    double v = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) v = fmax(v, fabs(a[i]));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int w = 0; w < int(blockDim.x >> 6); ++w) m = fmax(m, red[w]);
        out[0] = m;
    }
}

constexpr int SQ_MAX = 32;   // largest quadrature order

__device__ double block_sum256(double v, double* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < 4; ++w) s += red[w];
    return s;
}

__global__ __launch_bounds__(256) void sq_lanczos_kernel(int m, const double* C, int n_o,
                                                         const double* cmax, double* part) {
    extern __shared__ double sh[];
    double* q = sh;             // m
    double* qp = sh + m;        // m
    double* w = sh + 2 * m;     // m
    __shared__ double red[4];
    __shared__ double A[SQ_MAX * SQ_MAX], Vv[SQ_MAX * SQ_MAX];
    __shared__ int kdim;
    const int r = blockIdx.x, tid = threadIdx.x;
    for (int i = tid; i < m; i += 256) {
        q[i] = (i == r) ? 1.0 : 0.0;
        qp[i] = 0.0;
    }
    for (int i = tid; i < SQ_MAX * SQ_MAX; i += 256) A[i] = 0.0;
    if (tid == 0) kdim = n_o;
    __syncthreads();
    const double tiny = 1e-14 * fmax(cmax[0], 1e-300);
    double beta = 0.0;
    for (int k = 0; k < n_o; ++k) {
        // w = C q - beta q_prev
        for (int i = tid; i < m; i += 256) {
            double s = 0.0;
            for (int j = 0; j < m; ++j) s += C[i + int64_t(m) * j] * q[j];
            w[i] = s - beta * qp[i];
        }
        __syncthreads();
        double pa = 0.0;
        for (int i = tid; i < m; i += 256) pa += q[i] * w[i];
        const double alpha = block_sum256(pa, red);
        for (int i = tid; i < m; i += 256) w[i] -= alpha * q[i];
        if (tid == 0) A[k + SQ_MAX * k] = alpha;
        __syncthreads();
        if (k == n_o - 1) break;
        double pb = 0.0;
        for (int i = tid; i < m; i += 256) pb += w[i] * w[i];
        beta = sqrt(block_sum256(pb, red));
        if (!(beta > tiny)) {
            if (tid == 0) kdim = k + 1;
            __syncthreads();
            break;
        }
        for (int i = tid; i < m; i += 256) {
            qp[i] = q[i];
            q[i] = w[i] / beta;
        }
        if (tid == 0) {
            A[k + 1 + SQ_MAX * k] = beta;
            A[k + SQ_MAX * (k + 1)] = beta;
        }
        __syncthreads();
    }
    __syncthreads();
    // cyclic Jacobi on the kdim x kdim tridiagonal (one thread; kdim <= 32)
    if (tid == 0) {
        const int n = kdim;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) Vv[i + SQ_MAX * j] = (i == j) ? 1.0 : 0.0;
        for (int sweep = 0; sweep < 100; ++sweep) {
            double off = 0.0, dia = 0.0;
            for (int i = 0; i < n; ++i) {
                dia += A[i + SQ_MAX * i] * A[i + SQ_MAX * i];
                for (int j = i + 1; j < n; ++j) off += A[i + SQ_MAX * j] * A[i + SQ_MAX * j];
            }
            if (!(off > 1e-30 * dia)) break;
            for (int p = 0; p < n - 1; ++p)
                for (int qq = p + 1; qq < n; ++qq) {
                    const double apq = A[p + SQ_MAX * qq];
                    if (apq == 0.0) continue;
                    const double app = A[p + SQ_MAX * p], aqq = A[qq + SQ_MAX * qq];
                    const double theta = (aqq - app) / (2.0 * apq);
                    const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                    const double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
                    for (int k = 0; k < n; ++k) {   // A <- A G (columns p, q)
                        const double akp = A[k + SQ_MAX * p], akq = A[k + SQ_MAX * qq];
                        A[k + SQ_MAX * p] = c * akp - sn * akq;
                        A[k + SQ_MAX * qq] = sn * akp + c * akq;
                    }
                    for (int k = 0; k < n; ++k) {   // A <- G^T A (rows p, q)
                        const double apk = A[p + SQ_MAX * k], aqk = A[qq + SQ_MAX * k];
                        A[p + SQ_MAX * k] = c * apk - sn * aqk;
                        A[qq + SQ_MAX * k] = sn * apk + c * aqk;
                    }
                    for (int k = 0; k < n; ++k) {   // V <- V G
                        const double vkp = Vv[k + SQ_MAX * p], vkq = Vv[k + SQ_MAX * qq];
                        Vv[k + SQ_MAX * p] = c * vkp - sn * vkq;
                        Vv[k + SQ_MAX * qq] = sn * vkp + c * vkq;
                    }
                }
        }
        double e = 0.0;
        for (int t = 0; t < n; ++t) {
            const double lam = A[t + SQ_MAX * t], q0 = Vv[0 + SQ_MAX * t];
            e += q0 * q0 * (log1p(-lam) + lam);
        }
        part[r] = e;
    }
}

// out[0] = scale * sum_r part[r] in a fixed order (deterministic); info[0] = 0, or 1 if the
// sum is not finite
__global__ __launch_bounds__(256) void sq_sum_kernel(int m, const double* part, double scale,
                                                     double* out, int* info) {
    __shared__ double red[4];
    double v = 0.0;
    for (int i = threadIdx.x; i < m; i += 256) v += part[i];
    const double s = block_sum256(v, red);
    if (threadIdx.x == 0) {
        out[0] = scale * s;
        info[0] = isfinite(s) ? 0 : 1;
    }
}

}  // namespace

hipError_t launch_sq_energy(int m, const double* C, int n_o, double scale, double* work,
                            double* out, int* info, hipStream_t s) {
    if (n_o < 1 || n_o > SQ_MAX) return hipErrorInvalidValue;
    double* cmax = work;
    double* part = work + 1;
    hipLaunchKernelGGL(absmax_kernel, dim3(1), dim3(256), 0, s, int64_t(m) * m, C, cmax);
    const size_t sh = 3 * size_t(m) * sizeof(double);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(sq_lanczos_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(sh));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sq_lanczos_kernel, dim3(m), dim3(256), sh, s, m, C, n_o, cmax, part);
    hipLaunchKernelGGL(sq_sum_kernel, dim3(1), dim3(256), 0, s, m, part, scale, out, info);
    return hipGetLastError();
}


hipError_t launch_symmetrize(int m, double* C, hipStream_t s) {
    hipLaunchKernelGGL(symmetrize_kernel, dim3((m * m + 255) / 256), dim3(256), 0, s, m, C);
    return hipGetLastError();
}

hipError_t launch_chol_inv(int m, const double* M, double* L, double* T, int* info,
                           hipStream_t s) {
    const size_t lds = 2 * size_t(m) * m * sizeof(double);
    if (lds <= size_t(kSmallLdsBytes)) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(chol_inv_lds_kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(chol_inv_lds_kernel, dim3(1), dim3(SB), lds, s, m, M, L, T, info);
    } else {
        hipLaunchKernelGGL(chol_inv_kernel, dim3(1), dim3(SB), size_t(m) * sizeof(double), s, m,
                           M, L, T, info);
    }
    return hipGetLastError();
}

hipError_t launch_energy_logdet(int m, const double* C, double scale, double* work,
                                double* out, int* info, hipStream_t s) {
    const size_t lds = size_t(m) * m * sizeof(double);
    if (2 * lds <= size_t(kSmallLdsBytes)) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(energy_lds_kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(energy_lds_kernel, dim3(1), dim3(SB), lds, s, m, C, scale, out, info);
    } else {
        hipLaunchKernelGGL(energy_kernel, dim3(1), dim3(SB), size_t(m) * sizeof(double), s, m, C,
                           scale, work, out, info);
    }
    return hipGetLastError();
}

hipError_t launch_syevj(int m, const double* A, double* work, double* w, double* Y,
                        hipStream_t s) {
    const int np = (m + 1) / 2;
    const size_t sh = size_t(2 * np) * sizeof(double) + size_t(2 * np) * sizeof(int);
    hipLaunchKernelGGL(syevj_kernel, dim3(1), dim3(SB), sh, s, m, A, work, w, Y);
    return hipGetLastError();
}

hipError_t launch_drho(int64_t nd, int ns, int nvec, const double* psi, const double* x,
                       int stride, double* out, hipStream_t s) {
    const dim3 grid(unsigned((nd + 255) / 256), nvec);
    if (stride == 2)
        hipLaunchKernelGGL(drho_kernel<2>, grid, dim3(256), 0, s, nd, ns, psi, x, out);
    else
        hipLaunchKernelGGL(drho_kernel<1>, grid, dim3(256), 0, s, nd, ns, psi, x, out);
    return hipGetLastError();
}

hipError_t launch_grad_accum_d(int64_t nd, int ns, int nvec, const double* psi,
                               const double* eps, double omega, const double* coeff,
                               double2* dbuf, const double* coefk, const void* x, bool x_fp32,
                               double* grad, hipStream_t s) {
    const int S = ns * nvec;
    hipLaunchKernelGGL(grad_d_kernel, dim3((ns * S + 255) / 256), dim3(256), 0, s, ns, S, eps,
                       omega, coeff, dbuf);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 grid(unsigned((nd + 127) / 128)), block(128);
#define RPA_G(NSM)                                                                           \
    if (ns <= NSM) {                                                                         \
        if (x_fp32)                                                                          \
            hipLaunchKernelGGL((grad_kernel<float2, NSM>), grid, block, 0, s, nd, ns, nvec,  \
                               psi, dbuf, coefk, reinterpret_cast<const float2*>(x), grad);  \
        else                                                                                 \
            hipLaunchKernelGGL((grad_kernel<double2, NSM>), grid, block, 0, s, nd, ns, nvec, \
                               psi, dbuf, coefk, reinterpret_cast<const double2*>(x), grad); \
        return hipGetLastError();                                                            \
    }
    RPA_G(8) RPA_G(16) RPA_G(32) RPA_G(64) RPA_G(128)
#undef RPA_G
    return hipErrorInvalidValue;
}

hipError_t launch_scale(int64_t n, double a, double* x, hipStream_t s) {
    hipLaunchKernelGGL(scale_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, n, a, x);
    return hipGetLastError();
}

hipError_t launch_fill(int64_t n, double v, double* x, hipStream_t s) {
    hipLaunchKernelGGL(fill_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, n, v, x);
    return hipGetLastError();
}

__global__ void to_float_kernel(int64_t n, const double* __restrict__ src,
                                float* __restrict__ dst) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = float(src[i]);
}

hipError_t launch_to_float(int64_t n, const double* src, float* dst, hipStream_t s) {
    hipLaunchKernelGGL(to_float_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, n, src,
                       dst);
    return hipGetLastError();
}

hipError_t launch_copy(int64_t n, const double* src, double* dst, hipStream_t s) {
    hipLaunchKernelGGL(copy_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, n, src, dst);
    return hipGetLastError();
}

}  // namespace rpa
