// Internal declarations of the gfx950 RPA library: device helpers, kernel launchers and
// the workspace carver.  Everything here is private to the shared library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/rpa.h"

namespace rpa {

// ------------------------------------------------------------------ error plumbing
void set_error(const std::string& msg);

struct Status {
    int code = RPA_OK;
};

#define RPA_HIP(call)                                                              \
    do {                                                                           \
        hipError_t e_ = (call);                                                    \
        if (e_ != hipSuccess) {                                                    \
            ::rpa::set_error(std::string("HIP error '") + hipGetErrorString(e_) +  \
                             "' at " __FILE__ ":" + std::to_string(__LINE__));     \
            return RPA_EHIP;                                                       \
        }                                                                          \
    } while (0)

#define RPA_CHECK(rc)              \
    do {                           \
        int rc_ = (rc);            \
        if (rc_ < 0) return rc_;   \
    } while (0)

// ------------------------------------------------------------------ workspace carver
// Bump allocator over the caller's workspace.  With base == nullptr it only counts, so the
// size query and the real carving run the same code and always agree.
struct Carver {
    char* base = nullptr;
    size_t used = 0;
    template <typename T>
    T* take(size_t count) {
        used = (used + 255) & ~size_t(255);
        T* p = base ? reinterpret_cast<T*>(base + used) : nullptr;
        used += count * sizeof(T);
        return p;
    }
};

// ------------------------------------------------------------------ grid geometry
struct Grid {
    int n0, n1, n2;
    double h;
    int bc = 0;      // RPA_BC_PERIODIC or RPA_BC_DIRICHLET
    int64_t nd() const { return int64_t(n0) * n1 * n2; }
    bool periodic() const { return bc == 0; }
};

// 12th-order centred second-derivative weights w_0..w_6 (exact rationals, see fd_weights()).
void fd_weights(double w[7]);

// ------------------------------------------------------------------ kernel launchers
// All launchers enqueue on `s` and return hipError_t of the launch.

// Kronecker nu^{power/2}: 1D eigenbases (basis[3] device, n_a*n_a each, kappa[3] device n_a)
hipError_t launch_eigbasis_1d(int n, double h, double* U, double* kappa, hipStream_t s);
// Isolated box: eigenpairs of the Dirichlet -D2 (banded Toeplitz of the weights, n <= 4096
// not required small but work >= 3 n^2 doubles), kappa ascending, U[t + n a] = mode a.
hipError_t launch_eigbasis_1d_box(int n, double h, double* U, double* kappa, double* work,
                                  hipStream_t s);
hipError_t launch_kron_apply(const Grid& g, int power, int nvec, const double* in, double* out,
                             double* tmp, const double* Ux, const double* Uy, const double* Uz,
                             const double* kx, const double* ky, const double* kz,
                             hipStream_t s);
// Shifted-Laplacian preconditioner on nsys complex vectors stored as N_d x 2 nsys real
// columns (real and imaginary part of system t in columns 2t, 2t+1): out = K_t^{-1} in with
// K_t = -1/2 Lap_h + kshift[t].x - i kshift[t].y, through the same 1D eigenbases.
hipError_t launch_kron_precond(const Grid& g, int nsys, const double* in, double* out,
                               double* tmp, const double* Ux, const double* Uy, const double* Uz,
                               const double* kx, const double* ky, const double* kz,
                               const double2* kshift, hipStream_t s);

// Preconditioned COCG (Kronecker shifted-Laplacian preconditioner) on nsys systems, FP64,
// host-driven iterations of batched kernels (one workgroup per system for the stencil,
// reductions and updates; the preconditioner as Kronecker passes over all systems).  The
// complex vectors r, p, z, q live as N_d x 2 nsys real column blocks.  See pcocg.hip.
// Widest block of the block COCG solver.
constexpr int kMaxBlockWidth = 8;

struct PcocgLaunch {
    Grid g;
    int nsys, ns;
    // block COCG: width >= 2 (at most kMaxBlockWidth); the slots of block b are
    // boff[b] .. boff[b+1]-1 (device, nblk + 1 offsets); 0: every system on its own
    int width = 0, nblk = 0;
    const int* boff = nullptr;
    int* split = nullptr;   // device, nsys: per-block split state (at the block's first slot)
    bool kron = true;       // apply K^{-1} (false: the identity, block COCG only)
    const double* vloc;
    const double* eps;      // device, ns
    const double* omega_v;  // device, nsys / ns: frequency of trial vector j
    const int* order;       // device, nsys: slot t solves system order[t] (a permutation)
    const double2* kshift;  // device, nsys: (sigma, omega) of slot t's preconditioner
    double tol;
    int max_iter;
    const double2* rhs;     // nsys x N_d complex (interleaved): right-hand sides
    double2* x;             // nsys x N_d complex (interleaved): solutions
    double *r, *p, *z, *q, *tmp;   // N_d x 2 nsys each
    double2* rho;           // nsys (block COCG: nsys x kMaxBlockWidth)
    double* b2;             // nsys
    int *active, *iters, *status;  // nsys
    const double *Ux, *Uy, *Uz, *kx, *ky, *kz;
};
// Runs the whole solve (synchronises the stream every few iterations to test for the end).
hipError_t launch_pcocg(const PcocgLaunch& L, hipStream_t s);
// mean of V_loc into *out (device)
hipError_t launch_vloc_mean(int64_t nd, const double* vloc, double* out, hipStream_t s);

// Occupied projector: coeff[l + ns*s] = dV sum_r psi[r,l] psi[r,n(s)] u[r,j(s)],
// s = n + ns*j, for j in [0, nvec).  part: split-K partial buffer (nsplit*ns*ns*nvec).
hipError_t launch_proj_coeff(int64_t nd, int ns, int nvec, double dV, const double* psi,
                             const double* U, double* part, int nsplit, double* coeff,
                             hipStream_t s);
// r0[s][r] = -(psi[r,n] u[r,j] - sum_l psi[r,l] coeff[l,s]) written as complex (T = float or
// double) with zero imaginary part; if r64 != null the same value is also written there as
// complex float64 (the mixed path's float64 residual, which starts at the right-hand side).
template <typename T>
hipError_t launch_proj_rhs(int64_t nd, int ns, int nvec, const double* psi, const double* U,
                           const double* coeff, T* r0, double* r64, hipStream_t s);

// Batched COCG, one workgroup per system.  See cocg.hip for the layout.
struct CocgLaunch {
    Grid g;
    int nsys;              // systems in this launch
    int ns;                // orbitals (system s uses eps[s % ns])
    const double* vloc;    // N_d
    const double* eps;     // device, ns
    double omega;          // shift of every system unless omega_v is set
    const double* omega_v; // device, nsys / ns: frequency of trial vector j, or null
    const int* order;      // device, nsys: the systems to solve in dispatch order (a
                           // permutation of 0..nsys-1, or a subset of a larger launch's
                           // systems), or null
    double tol;
    int max_iter;
    void* r;               // nsys x N_d complex (T2)
    void* pa;              // nsys x N_d complex
    void* pb;              // nsys x N_d complex
    void* x;               // FP64: nsys x N_d real (complex if x_complex); mixed: complex FP64
    bool x_complex;
    int* iters;            // nsys
    int* status;           // nsys (0 ok, 1 not converged, 2 breakdown)
    bool fp32;             // mixed precision: state in complex64, reliable updates in FP64
    void* xlo;             // mixed: nsys x N_d complex64 partial solution
    double* rhi;           // mixed: nsys x N_d complex float64 residual (starts at the RHS)
    int* refinements;      // mixed: nsys (may be null)
    double refine_tol;     // mixed: residual drop that triggers a reliable update
    int refine_gap;        // mixed: fewest iterations between reliable updates
    const float* vloc32;   // mixed: V_loc in float32 for the complex64 sweeps (or null)
    double* b2;            // per system |b|^2: written by the mixed kernel, read by an
                           // FP64 continuation (x_accum) as its tolerance reference; or null
    bool x_accum;          // FP64 continuation: x is added to (not started at 0), and r
                           // starts at the true residual b - A x
};
hipError_t launch_cocg(const CocgLaunch& a, hipStream_t s);
// Host-only: whether the batched COCG kernel has a launch shape for this grid (a whole-plane
// variant of at most 3 columns per thread and 1024 threads, or row slabs of at least 12 rows
// with one column per thread), in FP64 and, with `mixed`, also in complex64.  No device call.
bool cocg_shape_exists(const Grid& g, bool mixed);

// Static device scratch of the allocation-free entry point (noalloc.hip): its size, and its
// device address on the current device (looked up once per device with hipGetSymbolAddress).
size_t noalloc_scratch_bytes();
int noalloc_scratch(void** out);

// Delta rho epilogue: out[r, j] = 4 sum_n psi[r,n] Re x[n + ns*j][r]; x is float64 with
// `stride` doubles per point (1: real parts only, 2: complex interleaved)
hipError_t launch_drho(int64_t nd, int ns, int nvec, const double* psi, const double* x,
                       int stride, double* out, hipStream_t s);

// Dense FP64 helpers on small N_r x N_r matrices and tall N_d x N_r blocks.
// G = A^T B (A: nd x m, B: nd x m, both column-major), G: m x m column-major; split-K.
hipError_t launch_gram(int64_t nd, int m, const double* A, const double* B, double* part,
                       int nsplit, double* G, hipStream_t s);
// Y = A * T (A: nd x m, T: m x m), Y may not alias A.
hipError_t launch_gemm_tall_small(int64_t nd, int m, const double* A, const double* T,
                                  double* Y, hipStream_t s);
// Symmetrise C <- (C + C^T)/2 (in place).
hipError_t launch_symmetrize(int m, double* C, hipStream_t s);
// Lower Cholesky of M (in place into L, upper part zeroed) then T = L^{-T} (upper).
// info[0] = 0 on success, k+1 if the k-th pivot is not positive.
hipError_t launch_chol_inv(int m, const double* M, double* L, double* T, int* info,
                           hipStream_t s);
// E = scale * (ln det(I - C) + tr C) via Cholesky of I - C; out[0] = E, info[0] as above.
hipError_t launch_energy_logdet(int m, const double* C, double scale, double* work,
                                double* out, int* info, hipStream_t s);
// Gauss spectral quadrature of order n_o (1..32): E = scale * sum_r e_r^T g(C) e_r by n_o
// Lanczos steps from each e_r; work >= m + 1 doubles; out[0] = E, info[0] = 0 (1: not finite).
hipError_t launch_sq_energy(int m, const double* C, int n_o, double scale, double* work,
                            double* out, int* info, hipStream_t s);
// Symmetric eigen-decomposition by cyclic Jacobi: A (m x m) copied to work; eigenvalues
// ascending into w, eigenvectors (columns) into Y if Y != nullptr.
hipError_t launch_syevj(int m, const double* A, double* work, double* w, double* Y,
                        hipStream_t s);

// Gradient epilogue for one block of systems (s = n + ns k):
// grad[r] += sum_s coefk[k] * 4 Re[(x_s + o_s)(r) x_s(r)],
// o_s = -sum_l psi[r,l] d[l,s],  d[l,s] = coeff[l,s] / (eps_l - eps_n - i omega) (into dbuf)
hipError_t launch_grad_accum_d(int64_t nd, int ns, int nvec, const double* psi,
                               const double* eps, double omega, const double* coeff,
                               double2* dbuf, const double* coefk, const void* x, bool x_fp32,
                               double* grad, hipStream_t s);
hipError_t launch_scale(int64_t n, double a, double* x, hipStream_t s);
hipError_t launch_copy(int64_t n, const double* src, double* dst, hipStream_t s);
hipError_t launch_fill(int64_t n, double v, double* x, hipStream_t s);
// dst[i] = float(src[i])
hipError_t launch_to_float(int64_t n, const double* src, float* dst, hipStream_t s);

}  // namespace rpa
