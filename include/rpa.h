/*
 * rpa.h -- C ABI of the MI355X (gfx950) library for the hot path of the real-space
 * DFPT random-phase-approximation correlation energy (Zhang, Shah, Pask, Chow,
 * Suryanarayana, arXiv:2504.01816).
 *
 * What the library computes (paper notation):
 *   E_c = (1/2pi) int_0^inf sum_{n<=N_r} [ln(1 - lambda_n(i w)) + lambda_n(i w)] dw      (Eq. 10)
 * with lambda the eigenvalues of chi0~ = nu^{1/2} chi0(i w) nu^{1/2} found by subspace
 * iteration (Algorithm 1), chi0 applied to a vector by density functional perturbation
 * theory (Eqs. 7-9): one complex-symmetric Sternheimer system
 *   (H - eps_n - i w) x = -(I - P_occ)(psi_n .* u),   H = -1/2 Lap_h + V_loc,
 * per occupied orbital n and trial vector u, solved by COCG (Sec. 3), and
 *   chi0 u = 4 sum_n Re(psi_n .* x_n)                                                     (Eq. 8).
 * nu^{1/2} is applied with the Kronecker product of the 1D finite-difference Laplacian
 * eigenbases (Sec. 3).
 *
 * Conventions shared by every call
 * --------------------------------
 * Grid: periodic n[0] x n[1] x n[2] points, spacing h (bohr), N_d = n0*n1*n2, flat index
 *   i = x + n0*(y + n1*z).  The Laplacian is the 12th-order centred stencil (radius 6).
 *   The GPU path needs n[2] >= 12 and n[0], n[1] >= 7.
 * Blocks of grid vectors are column-major N_d x k (column j contiguous, leading dim N_d).
 * Orbitals psi are grid-normalised: sum_r psi_m(r) psi_n(r) h^3 = delta_mn.
 * Memory: pointers documented "device" must be device (or managed) memory of the current
 *   HIP device; "host" pointers are ordinary host memory.  Every array is owned by the
 *   caller.  The library never allocates device memory: scratch space is the caller's
 *   workspace `ws` of `ws_bytes` bytes (device, 256-byte aligned), sized by
 *   rpa_workspace_size().  The library keeps no state between calls.
 * Streams: `stream` is a hipStream_t (NULL = the null stream).  All device work is
 *   enqueued on it.  Calls that return host values synchronise the stream before
 *   returning; the others return with the work enqueued.
 * Errors: every call returns an int: RPA_OK (0), a positive warning, or a negative error.
 *   Arguments are validated on the host before any device work; a validation failure
 *   leaves every output untouched.  No C++ exception crosses the ABI.
 *   rpa_last_error() gives a message for the most recent failure on the calling thread.
 */
#ifndef RPA_H_
#define RPA_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status codes */
#define RPA_OK            0
#define RPA_ENOTCONV      1   /* warning: some COCG system hit cocg_max_iter; results written */
#define RPA_ESUBCAP       2   /* warning: with ec_tol > 0, some frequency stopped at
                                 subspace_iters before its energy test held (Algorithm 1's
                                 epsilon_c test); results written, rpa_stats.subspace_capped
                                 counts those frequencies.  When RPA_ENOTCONV also holds, the
                                 call returns RPA_ENOTCONV. */
#define RPA_EINVAL       -1   /* bad argument (size, pointer, non-finite scalar, unsorted eps) */
#define RPA_EWORKSPACE   -2   /* workspace missing, misaligned or smaller than required */
#define RPA_EBREAKDOWN   -3   /* COCG bilinear form vanished before convergence */
#define RPA_ENOTPD       -4   /* Cholesky factor of R^T R (or of I - C) does not exist */
#define RPA_EHIP         -5   /* a HIP runtime call failed */
#define RPA_ENOTIMPL     -6   /* option combination not implemented */

/* ---------------------------------------------------------------- option values */
#define RPA_FP64          0   /* every step in float64 / complex128 */
#define RPA_MIXED         1   /* COCG state in complex64 with float64 residual refinement */

#define RPA_WARM          0   /* Sec. 3: the subspace of one frequency starts the next */
#define RPA_INDEPENDENT   1   /* every frequency starts from V0; all frequencies still
                                 iterating share one batched chi0 launch per iteration */

/* rpa_options.flags */
#define RPA_FLAG_PRECOND  1   /* Sternheimer solves by COCG preconditioned with the Kronecker
                                 shifted Laplacian K = -1/2 Lap_h + sigma_n - i omega,
                                 sigma_n = max(mean V_loc - eps_n, 1/2) (Sec. 3's
                                 Laplacian-based preconditioning); RPA_FP64 only */

#define RPA_BC_PERIODIC   0   /* periodic cell */
#define RPA_BC_DIRICHLET  1   /* isolated box (zero outside the grid) */

/* Operation selectors for rpa_workspace_size(). */
#define RPA_OP_COULOMB    0
#define RPA_OP_CHI0       1
#define RPA_OP_SUBSPACE   2
#define RPA_OP_ENERGY     3
#define RPA_OP_BACKWARD   4

/* One periodic cell with its ground state (the paper's input files, Sec. 3). */
typedef struct rpa_cell {
    int32_t n[3];          /* grid points along x, y, z */
    int32_t n_occ;         /* N_s, number of doubly occupied orbitals (>= 1) */
    double h;              /* grid spacing, > 0 */
    const double* v_loc;   /* device, N_d: local potential V_loc (Eq. 4 without V_xc, V_nl) */
    const double* psi;     /* device, N_d x N_s column-major, grid-normalised orbitals */
    const double* eps;     /* host, N_s orbital eigenvalues, strictly ascending */
    int32_t bc;            /* RPA_BC_PERIODIC (0, the crystal cells) or RPA_BC_DIRICHLET (1:
                              an isolated box, grid points at (i+1) h, every function zero
                              outside; nu = 4 pi (-Lap_h)^{-1} without a null space) */
} rpa_cell;

/* Solver options.  rpa_default_options() fills the defaults noted below. */
typedef struct rpa_options {
    int32_t precision;       /* RPA_FP64 (default) or RPA_MIXED */
    int32_t cocg_max_iter;   /* per system, default 5000 */
    double cocg_tol;         /* relative residual ||b' - A x|| / ||b'|| (Sec. 4.1), default 1e-8 */
    int32_t subspace_iters;  /* fixed count if ec_tol <= 0, else cap; default 50 */
    int32_t freq_mode;       /* RPA_WARM (default) or RPA_INDEPENDENT */
    double ec_tol;           /* relative energy threshold |E_k - E_{k-1}| <= ec_tol |E_k|;
                                <= 0 selects the fixed count; default 1e-8 */
    double refine_tol;       /* RPA_MIXED: relative drop of the complex64 residual between
                                float64 refinements (reliable updates), at least 8 iterations
                                apart except at the tolerance and the cap; default 0.3 */
    int32_t max_systems;     /* cap on Sternheimer systems in flight; 0 = as many as keep
                                the COCG state within 128 GiB (56 B per point and system in
                                FP64, 64 B mixed), shared by the cells of an rpa_energy call
                                in proportion to their uncapped state; the trial vectors are
                                split into chunks of equal size under the cap */
    int32_t flags;           /* 0 or RPA_FLAG_PRECOND */
    int32_t sq_order;        /* 0 (default): E_{c,m} from the Ritz values of C (exact
                                Rayleigh-Ritz, via ln det(I - C) + tr C); 1..32: Gauss
                                spectral quadrature of that order on C (Sec. 3, Algorithm 1:
                                Lanczos from every e_r, nodes and weights from the
                                tridiagonal).  The backward always differentiates the
                                Rayleigh-Ritz energy of the saved subspaces, which the SQ
                                energy converges to as the order grows. */
    int32_t cocg_block;      /* 0 or 1 (default): every Sternheimer system is solved on its
                                own.  2..8: block COCG (Sec. 3 names the block variant of
                                the solver): the systems of one orbital n and one frequency
                                share their matrix H - eps_n - i omega, so runs of up to
                                cocg_block consecutive trial vectors with equal frequency
                                (within one launch) are solved as one block with a shared
                                Krylov space; a column leaves its block when its relative
                                residual reaches cocg_tol.  With RPA_FLAG_PRECOND the block
                                iteration is preconditioned by the Kronecker shifted
                                Laplacian.  RPA_FP64 only (RPA_ENOTIMPL with RPA_MIXED);
                                the state is that of RPA_FLAG_PRECOND (112 B per point and
                                system). */
    double mixed_min_omega;  /* RPA_MIXED: trial vectors at frequencies below this (Ha) are
                                solved in FP64 (complex128 state) instead of complex64: near the
                                real axis the shifts approach the spectrum and the complex64
                                recurrences need more extra iterations than they save; 0 runs
                                every frequency in complex64.  Default 0.2. */
} rpa_options;

/* Counters accumulated by a call (added to the struct's current contents). */
typedef struct rpa_stats {
    int64_t cocg_iters_total;     /* sum over systems of COCG iterations (products with A) */
    int64_t cocg_systems;         /* Sternheimer systems solved */
    int32_t cocg_iters_max;       /* largest iteration count of one system */
    int32_t n_unconverged;        /* systems that hit cocg_max_iter */
    int32_t n_breakdown;          /* systems with a vanishing bilinear form */
    int32_t refinements;          /* float64 residual refinements (RPA_MIXED) */
    int32_t chi0_applies;         /* chi0 block-applies (one per subspace iteration) */
    int32_t subspace_iters_total; /* subspace iterations over all frequencies and cells */
    int64_t cocg_launches;        /* launches of the batched COCG kernel */
    double cocg_kernel_ms;        /* their summed duration, from HIP events recorded on the
                                     stream of each launch */
    double cocg_point_iters;      /* sum over systems of (COCG iterations x N_d) */
    int32_t fp64_fallbacks;       /* RPA_MIXED: systems that reached cocg_max_iter or broke
                                     down in complex64 and were solved on in FP64 from where
                                     they stopped, with the exact residual (up to
                                     cocg_max_iter further iterations); only a second cap or
                                     breakdown there counts in n_unconverged / n_breakdown */
    int32_t subspace_capped;      /* frequencies whose subspace iteration stopped at
                                     subspace_iters with ec_tol > 0 before
                                     |E_k - E_{k-1}| <= ec_tol |E_k| held (the energy
                                     reported is that of the last iterate) */
} rpa_stats;

/* Library version (major*10000 + minor*100 + patch). */
int rpa_version(void);
/* Static string for a status code. */
const char* rpa_error_string(int code);
/* Message for the most recent failure of a call on this thread ("" if none). */
const char* rpa_last_error(void);
/* Fill *opt with the defaults listed in rpa_options. Returns RPA_EINVAL for NULL. */
int rpa_default_options(rpa_options* opt);

/*
 * Workspace bytes needed by an operation (host-only arithmetic; no device access).
 *   op      one of RPA_OP_*
 *   ncell   number of cells (1 except for RPA_OP_ENERGY)
 *   cells   host array of ncell cells (only n, n_occ and h are read)
 *   nvec    host array of ncell block widths: nvec for COULOMB/CHI0, N_r otherwise
 *   nfreq   number of frequencies (BACKWARD, and ENERGY with RPA_INDEPENDENT, whose
 *           workspace holds every frequency's block; ignored otherwise)
 *   opt     options (NULL = defaults)
 *   bytes   host out
 */
int rpa_workspace_size(int32_t op, int32_t ncell, const rpa_cell* cells, const int32_t* nvec,
                       int32_t nfreq, const rpa_options* opt, size_t* bytes);

/*
 * out = nu^{power/2} in for power in {1, 2}, nu = 4 pi (-Lap_h)^+ (Eq. 5; pseudo-inverse on
 * the zero-mean subspace, so the constant mode maps to 0), applied by the Kronecker-product
 * scheme of Sec. 3: transforms with the 1D eigenbases of -D2 along x, y, z, a pointwise
 * scale by (4 pi / (kx + ky + kz))^{power/2}, and the inverse transforms.
 *   in, out  device, N_d x nvec column-major float64 (out may equal in)
 */
int rpa_apply_coulomb(const rpa_cell* cell, int32_t power, int32_t nvec, const double* in,
                      double* out, void* ws, size_t ws_bytes, void* stream);

/*
 * rpa_apply_coulomb without a workspace, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid allocation).
 * Same operation, arguments and results as rpa_apply_coulomb.  Its scratch space (the 1D
 * bases and the transform buffer) is a static 32 MiB device array inside the library: every
 * GPU the library runs on holds its own copy from the first call on that device until the
 * process ends.  The call allocates nothing and enqueues its work on `stream`; the vectors
 * are transformed in passes of as many columns as the scratch holds (one column needs about
 * 8 N_d bytes).  Every call on one GPU shares that GPU's array and leaves its contents there:
 * calls that overlap on one GPU (other streams, other host threads) race and must be
 * serialised by the caller.
 *   in, out  device, N_d x nvec column-major float64 (out may equal in)
 * Returns RPA_EWORKSPACE (with a message naming the sizes) when one column of the grid and
 * its bases exceed the 32 MiB scratch (from about 4 million grid points).
 */
int rpa_apply_coulomb_noalloc(const rpa_cell* cell, int32_t power, int32_t nvec, const double* in,
                              double* out, void* stream);

/*
 * out = chi0(i omega) in, one "chi0 block-apply" (Eqs. 7-9, Algorithm 1 inner loops):
 * for every orbital n and column u_j of `in`, b = psi_n .* u_j, c = h^3 Psi^T b,
 * b' = b - Psi c, COCG on (H - eps_n - i omega) x = -b' from x = 0 to
 * ||r|| <= cocg_tol ||b'||, then out_j = 4 sum_n psi_n .* Re(x_{n,j}).  No nu is applied.
 *   omega    > 0
 *   in, out  device, N_d x nvec column-major float64 (must not overlap)
 *   stats    host, optional (NULL)
 * Returns RPA_ENOTCONV if any system hit cocg_max_iter (out still written),
 * RPA_EBREAKDOWN on a COCG breakdown (RPA_MIXED: a complex64 breakdown is first restarted once
 * in FP64 from the current iterate).  Synchronises the stream (stats are host values).
 */
int rpa_apply_chi0(const rpa_cell* cell, double omega, int32_t nvec, const double* in,
                   double* out, const rpa_options* opt, rpa_stats* stats, void* ws,
                   size_t ws_bytes, void* stream);

/*
 * Algorithm 1's subspace iteration at one frequency omega with quadrature weight `weight`:
 * repeat { R = nu^{1/2} chi0 nu^{1/2} V; C = (V^T R + R^T V)/2;
 *          E = weight/(2 pi) sum_k g(mu_k), g(x) = ln(1-x)+x, mu = eig(C);
 *          M = R^T R = L L^T; V <- R L^{-T} }
 * for opt->subspace_iters iterations (ec_tol <= 0) or until |E_k - E_{k-1}| <= ec_tol |E_k|
 * (k >= 2, at most subspace_iters).  The energy uses the identity
 * sum_k g(mu_k) = ln det(I - C) + tr C (Cholesky of I - C, which is SPD since C <= 0).
 *   V         device, N_d x nr, in: orthonormal start block, out: block after the last
 *             orthonormalisation (the start of the next frequency in RPA_WARM mode)
 *   V_saved   device, N_d x nr, optional: the block that produced the reported energy
 *   C_out     device, nr x nr, optional: the C behind the reported energy
 *   ritz_out  host, nr, optional: eigenvalues of that C, ascending
 *   ec_out    host, required: the reported E_{c,m} (weight/(2 pi) included)
 *   n_iter    host, optional: subspace iterations taken
 * Synchronises the stream.
 */
int rpa_subspace_iter(const rpa_cell* cell, double omega, double weight, int32_t nr, double* V,
                      double* V_saved, double* C_out, double* ritz_out, double* ec_out,
                      int32_t* n_iter, const rpa_options* opt, rpa_stats* stats, void* ws,
                      size_t ws_bytes, void* stream);

/*
 * Full E_c (Eq. 10) for ncell independent cells: frequencies in the given order (highest
 * first, as in Algorithm 1), per-frequency subspace iteration as in rpa_subspace_iter,
 * E_c = sum_m E_{c,m}.  The start block V0 of each cell is orthonormalised once (Cholesky
 * step) and then used by the first frequency (RPA_WARM) or by every frequency
 * (RPA_INDEPENDENT).  In RPA_INDEPENDENT mode the frequencies advance together: each
 * subspace iteration packs the blocks of every frequency still iterating side by side and
 * applies chi0 to all of them in one batched COCG launch (each Sternheimer system with its
 * own shift), then the projection, energy and Cholesky-QR run per frequency; a frequency
 * leaves the batch when its own stopping test holds.  Per frequency the result equals the
 * warm-driver recurrence started from V0.
 *   omega, weight  host, nfreq each, omega > 0
 *   nr             host, ncell subspace sizes
 *   V0             host array of ncell device pointers, N_d x nr each (not modified)
 *   Vsave, Csave   optional host arrays of ncell device pointers: nfreq x (N_d x nr) and
 *                  nfreq x (nr x nr), the saved V_m and C_m per frequency (backward input)
 *   ec_out         host, ncell
 *   ec_freq_out    host, ncell x nfreq, optional
 *   iters_out      host, ncell x nfreq, optional: subspace iterations per frequency
 * Synchronises the stream.
 */
int rpa_energy(int32_t ncell, const rpa_cell* cells, const int32_t* nr, int32_t nfreq,
               const double* omega, const double* weight, const double* const* V0,
               double* const* Vsave, double* const* Csave, const rpa_options* opt,
               double* ec_out, double* ec_freq_out, int32_t* iters_out, rpa_stats* stats,
               void* ws, size_t ws_bytes, void* stream);

/*
 * grad_vloc = grad_ec * dE_c/dV_loc(r) with orbitals, eigenvalues and the saved subspaces
 * V_m held fixed: the plain partial derivative per grid value (not divided by h^3).
 * Per frequency: C_m = Y diag(mu) Y^T, W = V_m Y, u = nu^{1/2} W, Sternheimer solutions
 * x_{n,k} recomputed by COCG (the adjoint system equals the forward one because the
 * matrix is complex symmetric), o_{n,k} = -Psi [c_l / (eps_l - eps_n - i omega)]_l, and
 *   grad += weight_m/(2 pi) sum_k g'(mu_k) 4 sum_n Re[(x + o) .* x],  g'(x) = -x/(1-x).
 *   Vsave  device, nfreq x (N_d x nr); Csave device, nfreq x (nr x nr) (from rpa_energy)
 *   grad_vloc  device, N_d (overwritten)
 * Synchronises the stream.
 */
int rpa_energy_backward(const rpa_cell* cell, int32_t nfreq, const double* omega,
                        const double* weight, int32_t nr, const double* Vsave,
                        const double* Csave, double grad_ec, double* grad_vloc,
                        const rpa_options* opt, rpa_stats* stats, void* ws, size_t ws_bytes,
                        void* stream);

#ifdef __cplusplus
}
#endif
#endif /* RPA_H_ */
