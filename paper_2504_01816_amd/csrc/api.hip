// C ABI of the gfx950 RPA library: argument validation (host only), workspace carving and
// the drivers that sequence the kernels of the hot path.
//
// Call structure (Algorithm 1):
//   rpa_energy            for each cell: V <- chol-orthonormalise(V0); for each frequency
//                         (given order, highest first): rpa_subspace_iter
//   rpa_subspace_iter     repeat: u = nu^{1/2} V; D = chi0 u; R = nu^{1/2} D; C = sym(V^T R);
//                         E = W/(2pi)(ln det(I-C) + tr C); M = R^T R = L L^T; V = R L^{-T}
//   rpa_apply_chi0        per chunk of trial vectors: projector coefficients, projected
//                         right-hand sides, batched COCG (mixed precision: then the FP64
//                         continuation of systems stopped at the cap; RPA_FLAG_PRECOND: the
//                         preconditioned solver instead), Delta rho
//   rpa_energy_backward   per frequency: eig(C_m), W = V_m Y, u = nu^{1/2} W, COCG with the
//                         complex solutions kept, gradient accumulation
// In RPA_INDEPENDENT mode rpa_energy batches the frequencies still iterating into one chi0
// apply per subspace iteration; several cells run concurrently, one host thread and stream
// each, in their own workspace slices.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "internal.h"

namespace rpa {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

void fd_weights(double w[7]) {
    // Centred second-derivative weights of order 12 (radius 6):
    // w_p = 2 (-1)^{p+1} (6!)^2 / (p^2 (6-p)! (6+p)!),  w_0 = -2 sum_p w_p.
    w[0] = -5369.0 / 1800.0;
    w[1] = 12.0 / 7.0;
    w[2] = -15.0 / 56.0;
    w[3] = 10.0 / 189.0;
    w[4] = -1.0 / 112.0;
    w[5] = 2.0 / 1925.0;
    w[6] = -1.0 / 16632.0;
}

namespace {

constexpr int kVersion = 10100;

// RPA_MIXED: frequencies below this (Ha) solve in FP64.  Near the real axis the Sternheimer
// shifts come close to the spectrum and the complex64 recurrences lose conjugacy: measured on
// the 48^3 cell in subspace iterations after the first, complex64 needs 1.39x the FP64
// iterations at omega = 0.311 and 1.78x at 0.113 (2x and more at 0.0203), against a
// per-iteration saving of 1.45-1.6x: per block-apply complex64 is 1.04x faster at 0.311 and
// FP64 1.21x faster at 0.113 (on the 24^3 cell, where the kernel saves less per iteration,
// FP64 is already 1.16x faster at 0.311).  The 8-point rule has no node between 0.113 and
// 0.311.
constexpr double kMixedMinOmega = 0.2;

// RPA_MIXED: default relative drop of the complex64 residual that triggers a reliable update.
// Measured on the 48^3 cell (complex64 at every frequency): 0.3 takes 3-10% less time than 0.1
// at the three lowest frequencies (fewer iterations lost between updates), 0.01 and 0.001 take
// more; with the 8-iteration gap the fast systems at high frequency refine no more often.
constexpr double kRefineTol = 0.3;

struct Opts {
    int precision = RPA_FP64;
    int cocg_max_iter = 5000;
    double cocg_tol = 1e-8;
    int subspace_iters = 50;
    int freq_mode = RPA_WARM;
    double ec_tol = 1e-8;
    double refine_tol = kRefineTol;
    double mixed_min_omega = kMixedMinOmega;
    int max_systems = 0;
    int sq_order = 0;
    double state_budget = 0.0;   // bytes of COCG state per launch when max_systems = 0 (set
                                 // below: the library default, or a cell's share of it)
    bool precond = false;        // RPA_FLAG_PRECOND
    int block = 0;               // cocg_block: block COCG width (0, 1: off)
    // the host-driven solver (split vectors): preconditioned or block COCG
    bool host_driven() const { return precond || block >= 2; }
};

int fail(int code, const std::string& msg) {
    set_error(msg);
    return code;
}

int read_opts(const rpa_options* o, Opts* out) {
    Opts d;
    if (o) {
        d.precision = o->precision;
        d.cocg_max_iter = o->cocg_max_iter;
        d.cocg_tol = o->cocg_tol;
        d.subspace_iters = o->subspace_iters;
        d.freq_mode = o->freq_mode;
        d.ec_tol = o->ec_tol;
        d.refine_tol = o->refine_tol;
        d.mixed_min_omega = o->mixed_min_omega;
        d.max_systems = o->max_systems;
        d.sq_order = o->sq_order;
        if (o->flags & ~RPA_FLAG_PRECOND) return fail(RPA_EINVAL, "options.flags: unknown bits");
        d.precond = (o->flags & RPA_FLAG_PRECOND) != 0;
        d.block = o->cocg_block;
    }
    if (d.precision != RPA_FP64 && d.precision != RPA_MIXED)
        return fail(RPA_EINVAL, "options.precision must be RPA_FP64 or RPA_MIXED");
    if (d.cocg_max_iter < 1) return fail(RPA_EINVAL, "options.cocg_max_iter must be >= 1");
    if (!(d.cocg_tol > 0.0 && d.cocg_tol < 1.0))
        return fail(RPA_EINVAL, "options.cocg_tol must be in (0, 1)");
    if (d.subspace_iters < 1) return fail(RPA_EINVAL, "options.subspace_iters must be >= 1");
    if (d.freq_mode != RPA_WARM && d.freq_mode != RPA_INDEPENDENT)
        return fail(RPA_EINVAL, "options.freq_mode must be RPA_WARM or RPA_INDEPENDENT");
    if (!std::isfinite(d.ec_tol)) return fail(RPA_EINVAL, "options.ec_tol must be finite");
    if (!(d.refine_tol > 0.0 && d.refine_tol < 1.0))
        return fail(RPA_EINVAL, "options.refine_tol must be in (0, 1)");
    if (!(d.mixed_min_omega >= 0.0) || !std::isfinite(d.mixed_min_omega))
        return fail(RPA_EINVAL, "options.mixed_min_omega must be finite and >= 0");
    if (d.max_systems < 0) return fail(RPA_EINVAL, "options.max_systems must be >= 0");
    if (d.sq_order < 0 || d.sq_order > 32)
        return fail(RPA_EINVAL, "options.sq_order must be in [0, 32]");
    if (d.precond && d.precision != RPA_FP64)
        return fail(RPA_ENOTIMPL, "RPA_FLAG_PRECOND is implemented for RPA_FP64 only");
    if (d.block < 0 || d.block > kMaxBlockWidth)
        return fail(RPA_EINVAL, "options.cocg_block must be in [0, 8]");
    if (d.block >= 2 && d.precision != RPA_FP64)
        return fail(RPA_ENOTIMPL, "block COCG (options.cocg_block >= 2) is implemented for "
                                  "RPA_FP64 only");
    *out = d;
    return RPA_OK;
}

// Geometry-only validation (used by the workspace query).
int check_geometry(const rpa_cell* c) {
    if (!c) return fail(RPA_EINVAL, "cell is NULL");
    if (c->n[0] < 7 || c->n[1] < 7 || c->n[2] < 12)
        return fail(RPA_EINVAL, "grid must have n[0], n[1] >= 7 and n[2] >= 12");
    const int64_t nd = int64_t(c->n[0]) * c->n[1] * c->n[2];
    if (nd > (int64_t(1) << 26)) return fail(RPA_EINVAL, "grid larger than 2^26 points");
    if (int64_t(c->n[0]) * c->n[1] > 4096)
        return fail(RPA_EINVAL, "x-y plane larger than 4096 points");
    if (c->n[0] > 1024 || c->n[1] > 1024 || c->n[2] > 1024)
        return fail(RPA_EINVAL, "every axis must have at most 1024 points");
    if (!(c->h > 0.0) || !std::isfinite(c->h)) return fail(RPA_EINVAL, "h must be finite and > 0");
    if (c->n_occ < 1 || c->n_occ > 128 || c->n_occ >= nd)
        return fail(RPA_EINVAL, "n_occ must be in [1, 128] and below N_d");
    if (c->bc != RPA_BC_PERIODIC && c->bc != RPA_BC_DIRICHLET)
        return fail(RPA_EINVAL, "bc must be RPA_BC_PERIODIC or RPA_BC_DIRICHLET");
    return RPA_OK;
}

int check_cell(const rpa_cell* c) {
    RPA_CHECK(check_geometry(c));
    if (!c->v_loc || !c->psi) return fail(RPA_EINVAL, "cell v_loc / psi pointer is NULL");
    if (!c->eps) return fail(RPA_EINVAL, "cell eps (host) pointer is NULL");
    for (int i = 0; i < c->n_occ; ++i) {
        if (!std::isfinite(c->eps[i])) return fail(RPA_EINVAL, "eps has a non-finite value");
        if (i > 0 && !(c->eps[i] > c->eps[i - 1]))
            return fail(RPA_EINVAL, "eps must be strictly ascending");
    }
    return RPA_OK;
}

Grid grid_of(const rpa_cell* c) { return Grid{c->n[0], c->n[1], c->n[2], c->h, c->bc}; }

// The plain COCG kernel marches the x-y plane whole (at most 3072 points) or in row slabs of
// at least 12 rows; grids that fit neither are solved only by the host-driven solvers
// (RPA_FLAG_PRECOND or cocg_block >= 2), whose step kernel has a gathered fallback.
int check_solver_geometry(const rpa_cell* c, const Opts& o) {
    if (o.host_driven()) return RPA_OK;
    if (!cocg_shape_exists(grid_of(c), o.precision == RPA_MIXED))
        return fail(RPA_EINVAL, "no COCG launch shape fits this grid: the x-y plane exceeds "
                                "3072 points and n[1] has no divisor giving row slabs of at "
                                "least 12 rows and at most 1024 points (the preconditioned or "
                                "block solver accepts it)");
    return RPA_OK;
}

int check_ws(void* ws, size_t ws_bytes, size_t need) {
    if (need == 0) return RPA_OK;
    if (!ws) return fail(RPA_EWORKSPACE, "workspace pointer is NULL");
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0)
        return fail(RPA_EWORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < need)
        return fail(RPA_EWORKSPACE, "workspace too small: need " + std::to_string(need) +
                                        " bytes, got " + std::to_string(ws_bytes));
    return RPA_OK;
}

// ------------------------------------------------------------------ buffer plans
struct CoulombBuf {
    double *Ux, *Uy, *Uz, *kx, *ky, *kz, *tmp;
    double* ework;   // isolated box: 1D eigenproblem work, 3 n^2
};
void carve_coulomb(Carver& cv, const Grid& g, int nvec, CoulombBuf& b) {
    b.Ux = cv.take<double>(size_t(g.n0) * g.n0);
    b.Uy = cv.take<double>(size_t(g.n1) * g.n1);
    b.Uz = cv.take<double>(size_t(g.n2) * g.n2);
    b.kx = cv.take<double>(g.n0);
    b.ky = cv.take<double>(g.n1);
    b.kz = cv.take<double>(g.n2);
    b.tmp = cv.take<double>(size_t(g.nd()) * nvec);
    const size_t nm = size_t(std::max(g.n0, std::max(g.n1, g.n2)));
    b.ework = g.periodic() ? nullptr : cv.take<double>(3 * nm * nm);
}

struct Chi0Buf {
    int chunk;     // trial vectors per COCG launch
    int nsplit;    // split-K of the coefficient GEMM
    bool mixed;
    bool x_complex;
    double* eps;
    double* coeff;
    double* part;
    void *r, *pa, *pb, *x;
    void* xlo;      // mixed only
    double* rhi;    // mixed only: complex float64 residual
    double* b2;     // mixed only: |b|^2 per system, for the FP64 continuation
    float* vloc32;  // mixed only: V_loc in float32 for the complex64 sweeps
    int *iters, *status, *refine;
    double* omega_v;  // per trial vector of a chunk: its frequency
    int* order;       // per system of a chunk: dispatch order
    double2* dbuf;  // backward only
    // host-driven solver (RPA_FLAG_PRECOND or cocg_block >= 2): split complex vectors,
    // per-system scalars, the 1D eigenbases of the preconditioner and the mean of V_loc;
    // kron: apply K^{-1} (else the identity); block: block COCG width (0: single systems),
    // boff: slot offsets of the blocks, bsplit: their split states, prho: rho per slot
    // (block: 8 per slot)
    bool precond, kron;
    int block;
    int *boff, *bsplit;
    double *pr, *pp, *pz, *pq, *ptmp;
    double2 *prho, *kshift;
    double* pb2;
    int* pactive;
    double *Ux, *Uy, *Uz, *kx, *ky, *kz, *bwork, *vmean;
};

// Host side of a chi0 apply: the frequency of every trial vector, and per system (n + ns j
// over the whole apply) the iteration count of the previous apply of the same block, used to
// dispatch the longest solves first (-1: unknown).  Staging vectors stay alive until the
// stream synchronisation in tally().
struct Chi0Host {
    std::vector<double> omega;
    std::vector<int> hint;
    std::vector<double> om_chunk;
    std::vector<int> order, it, st, rf;
    std::vector<int> boff;            // block COCG: slot offsets of the blocks
    double vmean = 0.0;               // mean V_loc (preconditioner shifts)
    std::vector<double2> kshift;      // per system of a chunk: (sigma_n, omega_j)
    void reset(int ns, int nvec, double w) {
        omega.assign(nvec, w);
        hint.assign(size_t(ns) * nvec, -1);
    }
};

// Mixed precision: fewest COCG iterations between two reliable updates (besides the ones at the
// tolerance and at the cap).  Fast-converging systems would otherwise refine every two or three
// iterations (a refine_tol drop per step), each update a float64 sweep of about 90 B per
// point; at low frequency the updates are dozens of iterations apart and the gap does not
// bind.  Measured on the 48^3 cell: a gap of 12 is 3-4% faster from omega = 1.4 up, a gap of 16
// lets fast systems run 16 complex64 iterations past an update and breaks down at 49.4.
constexpr int kRefineGap = 8;

// COCG state kept in flight when the caller sets no cap: 128 GiB (under half the HBM of one
// MI355X), enough for every system of a block at 24^3 and 32^3 and for one frequency's block
// of 16384 systems at 48^3 in either precision.  Cells that run concurrently share it.
constexpr double kStateBudget = 128.0 * (1ull << 30);

// COCG state per point and system: FP64 r, p_a, p_b complex128 + x; mixed 64 B; the
// host-driven solver (preconditioned or block COCG) keeps r, p, z, q, a transform buffer, x
// and b: 112 B.
double state_bytes_per_point(const Opts& o) {
    return o.host_driven() ? 112.0 : (o.precision == RPA_MIXED ? 64.0 : 56.0);
}

// Trial vectors per COCG launch: as many as the cap allows, split into chunks of equal size
// (a small last chunk would leave most of the GPU idle).
int chunk_vectors(int64_t nd, int ns, int nvec, const Opts& o) {
    int cap = o.max_systems;
    if (cap == 0) {
        const double per_sys = double(nd) * state_bytes_per_point(o);
        const double budget = o.state_budget > 0.0 ? o.state_budget : kStateBudget;
        cap = int(std::min(double(1 << 30), std::floor(budget / per_sys)));
    }
    const int most = std::max(1, std::min(nvec, cap / ns));
    const int nch = (nvec + most - 1) / most;
    return (nvec + nch - 1) / nch;
}

int coeff_split(int64_t nd, int ns, int S) {
    const int tiles = ((ns + 63) / 64) * ((S + 63) / 64);
    int sp = std::max(1, 2048 / std::max(1, tiles));
    sp = int(std::min<int64_t>(sp, std::max<int64_t>(1, nd / 1024)));
    return sp;
}

void carve_chi0(Carver& cv, const Grid& g, int ns, int nvec, const Opts& o, bool x_complex,
                bool with_d, Chi0Buf& b) {
    b.chunk = chunk_vectors(g.nd(), ns, nvec, o);
    const int S = ns * b.chunk;
    const int64_t nd = g.nd();
    b.nsplit = coeff_split(nd, ns, S);
    b.mixed = (o.precision == RPA_MIXED);
    b.precond = o.host_driven();
    b.kron = o.precond;
    b.block = o.block >= 2 ? o.block : 0;
    // the mixed path keeps its solution as complex float64 (x_hi) for the true residual; the
    // preconditioned solver keeps it complex as well
    b.x_complex = x_complex || b.mixed || b.precond;
    const size_t cplx = b.mixed ? 8 : 16;
    b.eps = cv.take<double>(ns);
    b.coeff = cv.take<double>(size_t(ns) * S);
    b.part = cv.take<double>(size_t(b.nsplit) * ns * S);
    // mixed: r, p_a, p_b, x_lo (complex64) back to back, so that [r | p_a] and [p_b | x_lo]
    // each hold S x N_d complex128 values for the FP64 continuation of capped systems
    b.r = cv.take<char>(size_t(S) * nd * cplx);
    b.pa = cv.take<char>(size_t(S) * nd * cplx);
    b.pb = cv.take<char>(size_t(S) * nd * cplx);
    b.xlo = b.mixed ? cv.take<char>(size_t(S) * nd * 8) : nullptr;
    b.x = cv.take<char>(size_t(S) * nd * (b.x_complex ? 16 : 8));
    b.rhi = b.mixed ? cv.take<double>(2 * size_t(S) * nd) : nullptr;
    b.b2 = b.mixed ? cv.take<double>(S) : nullptr;
    b.vloc32 = b.mixed ? cv.take<float>(size_t(nd)) : nullptr;
    b.iters = cv.take<int>(S);
    b.status = cv.take<int>(S);
    b.refine = cv.take<int>(S);
    b.omega_v = cv.take<double>(b.chunk);
    b.order = cv.take<int>(S);
    b.dbuf = with_d ? cv.take<double2>(size_t(ns) * S) : nullptr;
    if (b.precond) {
        const size_t blk = 2 * size_t(S) * nd;
        b.pr = cv.take<double>(blk);
        b.pp = cv.take<double>(blk);
        b.pz = cv.take<double>(blk);
        b.pq = cv.take<double>(blk);
        b.ptmp = cv.take<double>(blk);
        b.prho = cv.take<double2>(size_t(S) * (b.block ? kMaxBlockWidth : 1));
        b.kshift = cv.take<double2>(S);
        b.pb2 = cv.take<double>(S);
        b.pactive = cv.take<int>(S);
        b.boff = b.block ? cv.take<int>(S + 1) : nullptr;
        b.bsplit = b.block ? cv.take<int>(S) : nullptr;
        b.Ux = cv.take<double>(size_t(g.n0) * g.n0);
        b.Uy = cv.take<double>(size_t(g.n1) * g.n1);
        b.Uz = cv.take<double>(size_t(g.n2) * g.n2);
        b.kx = cv.take<double>(g.n0);
        b.ky = cv.take<double>(g.n1);
        b.kz = cv.take<double>(g.n2);
        const size_t nm = size_t(std::max(g.n0, std::max(g.n1, g.n2)));
        b.bwork = g.periodic() ? nullptr : cv.take<double>(3 * nm * nm);
        b.vmean = cv.take<double>(1);
    } else {
        b.pr = b.pp = b.pz = b.pq = b.ptmp = nullptr;
        b.prho = b.kshift = nullptr;
        b.pb2 = nullptr;
        b.pactive = nullptr;
        b.boff = nullptr;
        b.bsplit = nullptr;
        b.Ux = b.Uy = b.Uz = b.kx = b.ky = b.kz = b.bwork = b.vmean = nullptr;
    }
}

int gram_split(int64_t nd, int m) {
    const int tiles = ((m + 63) / 64) * ((m + 63) / 64);
    int sp = std::max(1, 2048 / tiles);
    return int(std::min<int64_t>(sp, std::max<int64_t>(1, nd / 512)));
}

struct SubBuf {
    CoulombBuf cb;
    Chi0Buf xb;
    double *U, *D, *R, *C, *M, *L, *T, *part, *ework, *escal, *eigw, *eigwork;
    int* info;
    int gsplit;
};
void carve_sub(Carver& cv, const Grid& g, int ns, int nr, const Opts& o, SubBuf& b) {
    carve_coulomb(cv, g, nr, b.cb);
    carve_chi0(cv, g, ns, nr, o, false, false, b.xb);
    const size_t blk = size_t(g.nd()) * nr, sq = size_t(nr) * nr;
    b.U = cv.take<double>(blk);
    b.D = cv.take<double>(blk);
    b.R = cv.take<double>(blk);
    b.C = cv.take<double>(sq);
    b.M = cv.take<double>(sq);
    b.L = cv.take<double>(sq);
    b.T = cv.take<double>(sq);
    b.gsplit = gram_split(g.nd(), nr);
    b.part = cv.take<double>(size_t(b.gsplit) * sq);
    b.ework = cv.take<double>(2 * sq);
    b.escal = cv.take<double>(8);
    b.eigw = cv.take<double>(nr);
    b.eigwork = cv.take<double>(2 * sq);
    b.info = cv.take<int>(8);
}

struct EnergyBuf {
    SubBuf sb;
    double *Vstart, *Vcur;
};
void carve_energy(Carver& cv, const Grid& g, int ns, int nr, const Opts& o, EnergyBuf& b) {
    carve_sub(cv, g, ns, nr, o, b.sb);
    b.Vstart = cv.take<double>(size_t(g.nd()) * nr);
    b.Vcur = cv.take<double>(size_t(g.nd()) * nr);
}

// Independent frequencies batched: the blocks of all frequencies still iterating are packed
// side by side and go through one chi0 apply per subspace iteration.
struct BatchBuf {
    CoulombBuf cb;
    Chi0Buf xb;
    double *Vstart, *Vall, *P, *U, *D, *R;   // N_d x nr (Vstart), N_d x (nf nr) (the others)
    double *C, *M, *L, *T;                   // nr x nr per frequency
    double *part, *ework, *escal;
    int* info;
    int gsplit;
};
void carve_batch(Carver& cv, const Grid& g, int ns, int nr, int nf, const Opts& o, BatchBuf& b) {
    const int nall = nr * nf;
    carve_coulomb(cv, g, nall, b.cb);
    carve_chi0(cv, g, ns, nall, o, false, false, b.xb);
    const size_t blk = size_t(g.nd()) * nr, sq = size_t(nr) * nr;
    b.Vstart = cv.take<double>(blk);
    b.Vall = cv.take<double>(blk * nf);
    b.P = cv.take<double>(blk * nf);
    b.U = cv.take<double>(blk * nf);
    b.D = cv.take<double>(blk * nf);
    b.R = cv.take<double>(blk * nf);
    b.C = cv.take<double>(sq * nf);
    b.M = cv.take<double>(sq * nf);
    b.L = cv.take<double>(sq * nf);
    b.T = cv.take<double>(sq * nf);
    b.gsplit = gram_split(g.nd(), nr);
    b.part = cv.take<double>(size_t(b.gsplit) * sq);
    b.ework = cv.take<double>(2 * sq);
    b.escal = cv.take<double>(8 * size_t(nf));
    b.info = cv.take<int>(8 * size_t(nf));
}

struct BackBuf {
    CoulombBuf cb;
    Chi0Buf xb;
    double *W, *U, *Y, *mu, *eigwork, *coefk;
};
void carve_back(Carver& cv, const Grid& g, int ns, int nr, const Opts& o, BackBuf& b) {
    carve_coulomb(cv, g, nr, b.cb);
    carve_chi0(cv, g, ns, nr, o, true, true, b.xb);
    const size_t blk = size_t(g.nd()) * nr, sq = size_t(nr) * nr;
    b.W = cv.take<double>(blk);
    b.U = cv.take<double>(blk);
    b.Y = cv.take<double>(sq);
    b.mu = cv.take<double>(nr);
    b.eigwork = cv.take<double>(2 * sq);
    b.coefk = cv.take<double>(nr);
}

// ------------------------------------------------------------------ building blocks
int coulomb_setup(const Grid& g, const CoulombBuf& b, hipStream_t s) {
    if (g.periodic()) {
        RPA_HIP(launch_eigbasis_1d(g.n0, g.h, b.Ux, b.kx, s));
        RPA_HIP(launch_eigbasis_1d(g.n1, g.h, b.Uy, b.ky, s));
        RPA_HIP(launch_eigbasis_1d(g.n2, g.h, b.Uz, b.kz, s));
    } else {
        RPA_HIP(launch_eigbasis_1d_box(g.n0, g.h, b.Ux, b.kx, b.ework, s));
        RPA_HIP(launch_eigbasis_1d_box(g.n1, g.h, b.Uy, b.ky, b.ework, s));
        RPA_HIP(launch_eigbasis_1d_box(g.n2, g.h, b.Uz, b.kz, b.ework, s));
    }
    return RPA_OK;
}

int coulomb_apply(const Grid& g, const CoulombBuf& b, int power, int nvec, const double* in,
                  double* out, hipStream_t s) {
    RPA_HIP(launch_kron_apply(g, power, nvec, in, out, b.tmp, b.Ux, b.Uy, b.Uz, b.kx, b.ky, b.kz,
                              s));
    return RPA_OK;
}

struct SolveTally {
    int64_t iters_total = 0, systems = 0, launches = 0, refinements = 0;
    int iters_max = 0, unconv = 0, breakdown = 0, fallbacks = 0;
    int subcap = 0;   // frequencies stopped at subspace_iters before the energy test held
    double kernel_ms = 0.0, point_iters = 0.0;
};

// Events bracketing the COCG launches, created once per thread and device.
struct CocgTimer {
    hipEvent_t start = nullptr, stop = nullptr;
    int device = -1;
};
static thread_local CocgTimer g_timer;

// Destroy this thread's timing events (cell worker threads, before they end).
void release_timer() {
    if (g_timer.start) (void)hipEventDestroy(g_timer.start);
    if (g_timer.stop) (void)hipEventDestroy(g_timer.stop);
    g_timer = CocgTimer{};
}

int timer_events(hipEvent_t* a, hipEvent_t* b) {
    int dev = 0;
    RPA_HIP(hipGetDevice(&dev));
    if (g_timer.device != dev || !g_timer.start) {
        RPA_HIP(hipEventCreate(&g_timer.start));
        RPA_HIP(hipEventCreate(&g_timer.stop));
        g_timer.device = dev;
    }
    *a = g_timer.start;
    *b = g_timer.stop;
    return RPA_OK;
}

int tally(const Chi0Buf& b, int S, int64_t nd, SolveTally& t, Chi0Host& h, int64_t sys0,
          hipStream_t s) {
    h.it.assign(S, 0);
    h.st.assign(S, 0);
    h.rf.assign(S, 0);
    RPA_HIP(hipMemcpyAsync(h.it.data(), b.iters, sizeof(int) * S, hipMemcpyDeviceToHost, s));
    RPA_HIP(hipMemcpyAsync(h.st.data(), b.status, sizeof(int) * S, hipMemcpyDeviceToHost, s));
    if (b.mixed)
        RPA_HIP(hipMemcpyAsync(h.rf.data(), b.refine, sizeof(int) * S, hipMemcpyDeviceToHost, s));
    RPA_HIP(hipStreamSynchronize(s));
    hipEvent_t e0, e1;
    RPA_CHECK(timer_events(&e0, &e1));
    float ms = 0.0f;
    RPA_HIP(hipEventElapsedTime(&ms, e0, e1));
    t.kernel_ms += ms;
    t.launches += 1;
    for (int i = 0; i < S; ++i) {
        t.point_iters += double(h.it[i]) * double(nd);
        t.iters_total += h.it[i];
        t.iters_max = std::max(t.iters_max, h.it[i]);
        t.refinements += h.rf[i];
        t.unconv += (h.st[i] == 1);
        t.breakdown += (h.st[i] == 2);
        if (sys0 + i < int64_t(h.hint.size())) h.hint[sys0 + i] = h.it[i];
    }
    t.systems += S;
    return RPA_OK;
}

void add_stats(rpa_stats* st, const SolveTally& t) {
    if (!st) return;
    st->cocg_iters_total += t.iters_total;
    st->cocg_systems += t.systems;
    st->cocg_iters_max = std::max<int32_t>(st->cocg_iters_max, t.iters_max);
    st->n_unconverged += t.unconv;
    st->n_breakdown += t.breakdown;
    st->refinements += int32_t(t.refinements);
    st->cocg_launches += t.launches;
    st->cocg_kernel_ms += t.kernel_ms;
    st->cocg_point_iters += t.point_iters;
    st->fp64_fallbacks += t.fallbacks;
    st->subspace_capped += t.subcap;
}

// Dispatch order of the ns*nv systems of a chunk: the previous apply's iteration counts when
// every system has one, else an estimate of the difficulty, 1/|eps_top - eps_n + 0.05 + i w|
// (the shifted gap shrinks for orbitals near the top and for small frequencies); largest
// first, ties by system index.
void dispatch_order(const rpa_cell* cell, int nv, int64_t j0, Chi0Host& h) {
    const int ns = cell->n_occ, S = ns * nv;
    std::vector<double> key(S);
    bool have = true;
    for (int i = 0; i < S && have; ++i) have = h.hint[size_t(j0) * ns + i] >= 0;
    for (int i = 0; i < S; ++i) {
        if (have) {
            key[i] = double(h.hint[size_t(j0) * ns + i]);
        } else {
            const int n = i % ns;
            const double w = h.omega[j0 + i / ns];
            key[i] = 1.0 / std::hypot(cell->eps[ns - 1] - cell->eps[n] + 0.05, w);
        }
    }
    h.order.resize(S);
    for (int i = 0; i < S; ++i) h.order[i] = i;
    std::stable_sort(h.order.begin(), h.order.end(),
                     [&](int a, int b) { return key[a] > key[b]; });
}

// Block COCG: the systems n + ns j of one orbital n whose trial vectors j form a run of equal
// frequency are cut into blocks of at most `width` consecutive vectors from the start of the
// run; the blocks take consecutive slots, hardest first (the largest dispatch key of their
// members, from h.order), and h.order becomes the slot -> system map, h.boff the offsets.
void block_order(const rpa_cell* cell, int nv, int width, Chi0Host& h) {
    const int ns = cell->n_occ, S = ns * nv;
    std::vector<int> rank(S);
    for (int t = 0; t < S; ++t) rank[h.order[t]] = t;   // position in the dispatch order
    std::vector<std::vector<int>> blocks;
    for (int j = 0; j < nv;) {
        int e = j;
        while (e < nv && h.om_chunk[e] == h.om_chunk[j]) ++e;
        for (int a = j; a < e; a += width)
            for (int n = 0; n < ns; ++n) {
                std::vector<int> m;
                for (int jj = a; jj < std::min(e, a + width); ++jj) m.push_back(n + ns * jj);
                blocks.push_back(m);
            }
        j = e;
    }
    std::vector<int> first(blocks.size());
    for (size_t k = 0; k < blocks.size(); ++k) {
        first[k] = S;
        for (int i : blocks[k]) first[k] = std::min(first[k], rank[i]);
    }
    std::vector<int> bo(blocks.size());
    for (size_t k = 0; k < bo.size(); ++k) bo[k] = int(k);
    std::stable_sort(bo.begin(), bo.end(), [&](int a, int c) { return first[a] < first[c]; });
    h.order.clear();
    h.boff.assign(1, 0);
    for (int k : bo) {
        for (int i : blocks[k]) h.order.push_back(i);
        h.boff.push_back(int(h.order.size()));
    }
}

// Whether trial vectors at frequency w solve in FP64 although the buffers are mixed.
bool fp64_in_mixed(const Chi0Buf& b, const Opts& o, double w) {
    return b.mixed && w < o.mixed_min_omega;
}

// Solve the Sternheimer systems of the trial vectors j0 .. j0+nv-1 (columns of U, which
// points at column j0), each at its own frequency h.omega[j].  With mixed buffers and
// fp64_run, the run solves in FP64 inside the mixed state: the complex128 residual goes in
// r_hi, the two complex128 direction vectors in [r | p_a] and [p_b | x_lo] (as for the
// continuation of capped systems), the solution in the x_hi buffer: complex if x_complex,
// else only its real part, packed as in the FP64 path (what Delta rho reads).
int solve_chunk(const rpa_cell* cell, const Grid& g, const Opts& o, const Chi0Buf& b,
                const double* U, int64_t j0, int nv, bool x_complex, Chi0Host& h,
                hipStream_t s, bool fp64_run = false) {
    const int ns = cell->n_occ;
    const int64_t nd = g.nd();
    const double dV = g.h * g.h * g.h;
    RPA_HIP(launch_proj_coeff(nd, ns, nv, dV, cell->psi, U, b.part, b.nsplit, b.coeff, s));
    if (b.mixed && fp64_run) {
        RPA_HIP(launch_proj_rhs<double>(nd, ns, nv, cell->psi, U, b.coeff, b.rhi, nullptr, s));
    } else if (b.mixed) {
        RPA_HIP(launch_proj_rhs<float>(nd, ns, nv, cell->psi, U, b.coeff,
                                       reinterpret_cast<float*>(b.r), b.rhi, s));
        RPA_HIP(launch_to_float(nd, cell->v_loc, b.vloc32, s));
    }
    else
        RPA_HIP(launch_proj_rhs<double>(nd, ns, nv, cell->psi, U, b.coeff,
                                        reinterpret_cast<double*>(b.r), nullptr, s));
    h.om_chunk.assign(h.omega.begin() + j0, h.omega.begin() + j0 + nv);
    if (b.precond) {
        // slots in dispatch order (longest solve first), so the systems still iterating stay
        // in a prefix of the slots that the preconditioner passes cover
        dispatch_order(cell, nv, j0, h);
        if (b.block) block_order(cell, nv, b.block, h);
        RPA_HIP(hipMemcpyAsync(b.omega_v, h.om_chunk.data(), sizeof(double) * nv,
                               hipMemcpyHostToDevice, s));
        RPA_HIP(hipMemcpyAsync(b.order, h.order.data(), sizeof(int) * ns * nv,
                               hipMemcpyHostToDevice, s));
        if (b.block)
            RPA_HIP(hipMemcpyAsync(b.boff, h.boff.data(), sizeof(int) * h.boff.size(),
                                   hipMemcpyHostToDevice, s));
        h.kshift.resize(size_t(ns) * nv);
        for (int t = 0; t < ns * nv; ++t) {
            const int i = h.order[t];
            h.kshift[t] = double2{std::max(h.vmean - cell->eps[i % ns], 0.5), h.om_chunk[i / ns]};
        }
        RPA_HIP(hipMemcpyAsync(b.kshift, h.kshift.data(), sizeof(double2) * ns * nv,
                               hipMemcpyHostToDevice, s));
        PcocgLaunch P{};
        P.g = g;
        P.nsys = ns * nv;
        P.ns = ns;
        P.vloc = cell->v_loc;
        P.eps = b.eps;
        P.omega_v = b.omega_v;
        P.order = b.order;
        P.kshift = b.kshift;
        P.width = b.block;
        P.nblk = b.block ? int(h.boff.size()) - 1 : 0;
        P.boff = b.boff;
        P.split = b.bsplit;
        P.kron = b.kron;
        P.tol = o.cocg_tol;
        P.max_iter = o.cocg_max_iter;
        P.rhs = reinterpret_cast<const double2*>(b.r);
        P.x = reinterpret_cast<double2*>(b.x);
        P.r = b.pr;
        P.p = b.pp;
        P.z = b.pz;
        P.q = b.pq;
        P.tmp = b.ptmp;
        P.rho = b.prho;
        P.b2 = b.pb2;
        P.active = b.pactive;
        P.iters = b.iters;
        P.status = b.status;
        P.Ux = b.Ux;
        P.Uy = b.Uy;
        P.Uz = b.Uz;
        P.kx = b.kx;
        P.ky = b.ky;
        P.kz = b.kz;
        hipEvent_t e0, e1;
        RPA_CHECK(timer_events(&e0, &e1));
        RPA_HIP(hipEventRecord(e0, s));
        RPA_HIP(launch_pcocg(P, s));
        RPA_HIP(hipEventRecord(e1, s));
        return RPA_OK;
    }
    dispatch_order(cell, nv, j0, h);
    RPA_HIP(hipMemcpyAsync(b.omega_v, h.om_chunk.data(), sizeof(double) * nv,
                           hipMemcpyHostToDevice, s));
    RPA_HIP(hipMemcpyAsync(b.order, h.order.data(), sizeof(int) * ns * nv, hipMemcpyHostToDevice,
                           s));
    CocgLaunch L{};
    L.g = g;
    L.nsys = ns * nv;
    L.ns = ns;
    L.vloc = cell->v_loc;
    L.eps = b.eps;
    L.omega = h.om_chunk[0];
    L.omega_v = b.omega_v;
    L.order = b.order;
    L.tol = o.cocg_tol;
    L.max_iter = o.cocg_max_iter;
    L.r = b.r;
    L.pa = b.pa;
    L.pb = b.pb;
    L.x = b.x;
    L.x_complex = x_complex;
    L.iters = b.iters;
    L.status = b.status;
    L.fp32 = b.mixed;
    if (b.mixed && fp64_run) {
        L.r = b.rhi;
        L.pa = b.r;
        L.pb = b.pb;
        L.x_complex = x_complex;
        L.fp32 = false;
        L.refinements = b.refine;      // written as 0 by the FP64 kernel
        hipEvent_t e0, e1;
        RPA_CHECK(timer_events(&e0, &e1));
        RPA_HIP(hipEventRecord(e0, s));
        RPA_HIP(launch_cocg(L, s));
        RPA_HIP(hipEventRecord(e1, s));
        return RPA_OK;
    }
    L.xlo = b.xlo;
    L.rhi = b.rhi;
    L.refinements = b.refine;
    L.refine_tol = o.refine_tol;
    L.refine_gap = kRefineGap;
    L.vloc32 = b.vloc32;
    L.b2 = b.b2;
    hipEvent_t e0, e1;
    RPA_CHECK(timer_events(&e0, &e1));
    RPA_HIP(hipEventRecord(e0, s));
    RPA_HIP(launch_cocg(L, s));
    RPA_HIP(hipEventRecord(e1, s));
    return RPA_OK;
}

// Preconditioned solver: the 1D eigenbases of the shifted Laplacian (as for nu^{1/2}) and
// the mean of V_loc for the shifts sigma_n = max(mean V_loc - eps_n, 1/2).
int precond_setup(const rpa_cell* cell, const Grid& g, const Chi0Buf& b, Chi0Host& h,
                  hipStream_t s) {
    if (!b.precond) return RPA_OK;
    if (g.periodic()) {
        RPA_HIP(launch_eigbasis_1d(g.n0, g.h, b.Ux, b.kx, s));
        RPA_HIP(launch_eigbasis_1d(g.n1, g.h, b.Uy, b.ky, s));
        RPA_HIP(launch_eigbasis_1d(g.n2, g.h, b.Uz, b.kz, s));
    } else {
        RPA_HIP(launch_eigbasis_1d_box(g.n0, g.h, b.Ux, b.kx, b.bwork, s));
        RPA_HIP(launch_eigbasis_1d_box(g.n1, g.h, b.Uy, b.ky, b.bwork, s));
        RPA_HIP(launch_eigbasis_1d_box(g.n2, g.h, b.Uz, b.kz, b.bwork, s));
    }
    RPA_HIP(launch_vloc_mean(g.nd(), cell->v_loc, b.vmean, s));
    RPA_HIP(hipMemcpyAsync(&h.vmean, b.vmean, sizeof(double), hipMemcpyDeviceToHost, s));
    RPA_HIP(hipStreamSynchronize(s));
    return RPA_OK;
}

// Mixed precision: the systems of a chunk that stopped at the iteration cap or at a breakdown
// of the complex64 recurrence (it can lose conjugacy on the most ill-conditioned shifts) are
// solved on in FP64 from where they stopped, once (the restart of a broken-down COCG from its
// current iterate and true residual): the mixed kernel leaves x_hi and the exact
// r_hi = b - A x_hi, and the FP64 kernel solves A e = r_hi into x_hi += e to |r| <= tol |b|,
// with [r | p_a] and [p_b | x_lo] of the mixed state as its two complex128 direction buffers.
// Only those systems are launched (the dispatch list is their indices); a second breakdown or
// the cap in FP64 is reported.  Needs the host copy of the statuses from tally().
int continue_capped(const rpa_cell* cell, const Grid& g, const Opts& o, const Chi0Buf& b,
                    int nv, Chi0Host& h, SolveTally& t, hipStream_t s) {
    if (!b.mixed) return RPA_OK;
    const int S = cell->n_occ * nv;
    std::vector<int> capped;
    for (int i = 0; i < S; ++i)
        if (h.st[i] == 1 || h.st[i] == 2) capped.push_back(i);
    if (capped.empty()) return RPA_OK;
    RPA_HIP(hipMemcpyAsync(b.order, capped.data(), sizeof(int) * capped.size(),
                           hipMemcpyHostToDevice, s));
    CocgLaunch L{};
    L.g = g;
    L.nsys = int(capped.size());
    L.ns = cell->n_occ;
    L.vloc = cell->v_loc;
    L.eps = b.eps;
    L.omega = h.om_chunk[0];
    L.omega_v = b.omega_v;
    L.order = b.order;
    L.tol = o.cocg_tol;
    L.max_iter = o.cocg_max_iter;
    L.r = b.rhi;
    L.pa = b.r;
    L.pb = b.pb;
    L.x = b.x;
    L.x_complex = true;
    L.iters = b.iters;
    L.status = b.status;
    L.fp32 = false;
    L.b2 = b.b2;
    L.x_accum = true;
    hipEvent_t e0, e1;
    RPA_CHECK(timer_events(&e0, &e1));
    RPA_HIP(hipEventRecord(e0, s));
    RPA_HIP(launch_cocg(L, s));
    RPA_HIP(hipEventRecord(e1, s));
    std::vector<int> it(S), st(S);
    RPA_HIP(hipMemcpyAsync(it.data(), b.iters, sizeof(int) * S, hipMemcpyDeviceToHost, s));
    RPA_HIP(hipMemcpyAsync(st.data(), b.status, sizeof(int) * S, hipMemcpyDeviceToHost, s));
    RPA_HIP(hipStreamSynchronize(s));
    float ms = 0.0f;
    RPA_HIP(hipEventElapsedTime(&ms, e0, e1));
    t.kernel_ms += ms;
    t.launches += 1;
    t.fallbacks += int(capped.size());
    for (int i : capped) {
        t.point_iters += double(it[i]) * double(g.nd());
        t.iters_total += it[i];
        t.iters_max = std::max(t.iters_max, h.it[i] + it[i]);
        // counted by tally() from the mixed stage
        if (h.st[i] == 1)
            t.unconv -= 1;
        else
            t.breakdown -= 1;
        t.unconv += (st[i] == 1);
        t.breakdown += (st[i] == 2);
    }
    return RPA_OK;
}

// chi0 on nvec trial vectors, vector j at frequency h.omega[j].
int chi0_apply(const rpa_cell* cell, const Grid& g, int nvec, const double* in, double* out,
               const Opts& o, const Chi0Buf& b, Chi0Host& h, SolveTally& t, hipStream_t s) {
    const int ns = cell->n_occ;
    const int64_t nd = g.nd();
    RPA_HIP(hipMemcpyAsync(b.eps, cell->eps, sizeof(double) * ns, hipMemcpyHostToDevice, s));
    RPA_CHECK(precond_setup(cell, g, b, h, s));
    // launches of at most b.chunk vectors; with mixed buffers a launch also keeps to one
    // precision (vectors below mixed_min_omega solve in FP64)
    for (int j0 = 0; j0 < nvec;) {
        const bool f64 = fp64_in_mixed(b, o, h.omega[j0]);
        int nv = 1;
        while (nv < b.chunk && j0 + nv < nvec && fp64_in_mixed(b, o, h.omega[j0 + nv]) == f64) ++nv;
        RPA_CHECK(solve_chunk(cell, g, o, b, in + nd * j0, j0, nv, false, h, s, f64));
        RPA_CHECK(tally(b, ns * nv, nd, t, h, int64_t(j0) * ns, s));
        if (!f64) RPA_CHECK(continue_capped(cell, g, o, b, nv, h, t, s));
        // an FP64 run in mixed buffers leaves the real part packed (solve_chunk)
        RPA_HIP(launch_drho(nd, ns, nv, cell->psi, reinterpret_cast<const double*>(b.x),
                            (b.x_complex && !f64) ? 2 : 1, out + nd * j0, s));
        j0 += nv;
    }
    return RPA_OK;
}

int solve_status(const SolveTally& t) {
    if (t.breakdown) return fail(RPA_EBREAKDOWN, std::to_string(t.breakdown) +
                                                     " COCG system(s) broke down");
    if (t.unconv) {
        set_error(std::to_string(t.unconv) + " COCG system(s) hit cocg_max_iter");
        return RPA_ENOTCONV;
    }
    if (t.subcap) {
        set_error(std::to_string(t.subcap) + " frequency(ies) stopped at subspace_iters before "
                  "the energy test held");
        return RPA_ESUBCAP;
    }
    return RPA_OK;
}

// Algorithm 1's stopping test after subspace iteration k at one frequency: a fixed count when
// ec_tol <= 0, else |E_k - E_{k-1}| <= ec_tol |E_k| (k >= 2) or the cap.  *capped is set when
// the cap stops an iteration whose energy test has not held.
bool subspace_stop(const Opts& o, int k, double E, double Eprev, bool* capped) {
    *capped = false;
    if (o.ec_tol <= 0.0) return k >= o.subspace_iters;
    const bool met = k >= 2 && std::fabs(E - Eprev) <= o.ec_tol * std::fabs(E);
    if (met) return true;
    if (k >= o.subspace_iters) {
        *capped = true;
        return true;
    }
    return false;
}

// Orthonormalise R into V: M = R^T R = L L^T, V = R L^{-T}.
int chol_orthonormalize(const Grid& g, int nr, const double* R, double* V, SubBuf& b,
                        hipStream_t s) {
    const int64_t nd = g.nd();
    RPA_HIP(launch_gram(nd, nr, R, R, b.part, b.gsplit, b.M, s));
    RPA_HIP(launch_chol_inv(nr, b.M, b.L, b.T, b.info, s));
    int info = 0;
    RPA_HIP(hipMemcpyAsync(&info, b.info, sizeof(int), hipMemcpyDeviceToHost, s));
    RPA_HIP(hipStreamSynchronize(s));
    if (info != 0)
        return fail(RPA_ENOTPD, "Cholesky of R^T R failed at column " + std::to_string(info));
    RPA_HIP(launch_gemm_tall_small(nd, nr, R, b.T, V, s));
    return RPA_OK;
}

struct SubResult {
    double E = 0.0;
    int n_iter = 0;
};

int subspace_iter(const rpa_cell* cell, const Grid& g, double omega, double weight, int nr,
                  double* V, double* V_saved, double* C_out, double* ritz_out, const Opts& o,
                  SubBuf& b, SolveTally& t, rpa_stats* stats, SubResult& res, hipStream_t s,
                  bool coulomb_ready) {
    const int64_t nd = g.nd();
    if (!coulomb_ready) RPA_CHECK(coulomb_setup(g, b.cb, s));
    double Eprev = 0.0, E = 0.0;
    int k = 0;
    Chi0Host h;
    h.reset(cell->n_occ, nr, omega);
    for (;;) {
        ++k;
        RPA_CHECK(coulomb_apply(g, b.cb, 1, nr, V, b.U, s));
        RPA_CHECK(chi0_apply(cell, g, nr, b.U, b.D, o, b.xb, h, t, s));
        RPA_CHECK(coulomb_apply(g, b.cb, 1, nr, b.D, b.R, s));
        RPA_HIP(launch_gram(nd, nr, V, b.R, b.part, b.gsplit, b.C, s));
        RPA_HIP(launch_symmetrize(nr, b.C, s));
        if (o.sq_order > 0)
            RPA_HIP(launch_sq_energy(nr, b.C, o.sq_order, weight / (2.0 * M_PI), b.ework, b.escal,
                                     b.info, s));
        else
            RPA_HIP(launch_energy_logdet(nr, b.C, weight / (2.0 * M_PI), b.ework, b.escal, b.info, s));
        int info = 0;
        RPA_HIP(hipMemcpyAsync(&E, b.escal, sizeof(double), hipMemcpyDeviceToHost, s));
        RPA_HIP(hipMemcpyAsync(&info, b.info, sizeof(int), hipMemcpyDeviceToHost, s));
        RPA_HIP(hipStreamSynchronize(s));
        if (stats) {
            stats->chi0_applies += 1;
            stats->subspace_iters_total += 1;
        }
        if (info != 0 || !std::isfinite(E)) {
            // C should be negative semidefinite; if it is not, name the likely cause
            if (t.breakdown)
                return fail(RPA_EBREAKDOWN, "COCG breakdown in " + std::to_string(t.breakdown) +
                                                " system(s); I - C not positive definite");
            if (t.unconv)
                return fail(RPA_ENOTPD, std::to_string(t.unconv) + " COCG system(s) hit "
                                        "cocg_max_iter; I - C not positive definite");
            return fail(info != 0 ? RPA_ENOTPD : RPA_EINVAL,
                        info != 0 ? "I - C is not positive definite" : "non-finite subspace energy");
        }
        if (V_saved) RPA_HIP(launch_copy(nd * nr, V, V_saved, s));
        if (C_out) RPA_HIP(launch_copy(int64_t(nr) * nr, b.C, C_out, s));
        RPA_CHECK(chol_orthonormalize(g, nr, b.R, V, b, s));
        bool capped = false;
        const bool stop = subspace_stop(o, k, E, Eprev, &capped);
        Eprev = E;
        if (capped) t.subcap += 1;
        if (stop) break;
    }
    if (ritz_out) {
        // eigenvalues of the C behind the reported energy (still in b.C)
        RPA_HIP(launch_syevj(nr, b.C, b.eigwork, b.eigw, nullptr, s));
        RPA_HIP(hipMemcpyAsync(ritz_out, b.eigw, sizeof(double) * nr, hipMemcpyDeviceToHost, s));
        RPA_HIP(hipStreamSynchronize(s));
    }
    res.E = E;
    res.n_iter = k;
    return RPA_OK;
}


// E_c of one cell with every frequency started from V0 and all frequencies still iterating
// advanced together (one chi0 apply over their packed blocks per subspace iteration, each
// trial vector at its own frequency).  Each frequency stops by the same test as the warm
// driver.
int energy_batched(const rpa_cell* cell, int nr, int nfreq, const double* omega,
                   const double* weight, const double* V0, double* Vsave, double* Csave,
                   const Opts& o, BatchBuf& b, SolveTally& t, rpa_stats* stats, double* ec,
                   double* ec_freq, int32_t* iters, hipStream_t s) {
    const Grid g = grid_of(cell);
    const int64_t nd = g.nd();
    const int ns = cell->n_occ;
    const size_t blk = size_t(nd) * nr, sq = size_t(nr) * nr;
    RPA_CHECK(coulomb_setup(g, b.cb, s));
    // V0 -> orthonormal start (Cholesky-QR, as in the warm driver)
    {
        RPA_HIP(launch_gram(nd, nr, V0, V0, b.part, b.gsplit, b.M, s));
        RPA_HIP(launch_chol_inv(nr, b.M, b.L, b.T, b.info, s));
        int info = 0;
        RPA_HIP(hipMemcpyAsync(&info, b.info, sizeof(int), hipMemcpyDeviceToHost, s));
        RPA_HIP(hipStreamSynchronize(s));
        if (info != 0) return fail(RPA_ENOTPD, "Cholesky of V0^T V0 failed");
        RPA_HIP(launch_gemm_tall_small(nd, nr, V0, b.T, b.Vstart, s));
    }
    for (int f = 0; f < nfreq; ++f) RPA_HIP(launch_copy(int64_t(blk), b.Vstart, b.Vall + f * blk, s));
    std::vector<int> active(nfreq), k(nfreq, 0);
    for (int f = 0; f < nfreq; ++f) active[f] = f;
    std::vector<double> E(nfreq, 0.0), Eprev(nfreq, 0.0);
    std::vector<std::vector<int>> hintf(nfreq, std::vector<int>(size_t(ns) * nr, -1));
    std::vector<double> escal(8 * size_t(nfreq));
    std::vector<int> info(8 * size_t(nfreq));
    Chi0Host h;
    while (!active.empty()) {
        const int na = int(active.size()), ncol = na * nr;
        h.omega.resize(ncol);
        h.hint.resize(size_t(ns) * ncol);
        for (int a = 0; a < na; ++a) {
            const int f = active[a];
            RPA_HIP(launch_copy(int64_t(blk), b.Vall + f * blk, b.P + a * blk, s));
            for (int j = 0; j < nr; ++j) h.omega[size_t(a) * nr + j] = omega[f];
            std::copy(hintf[f].begin(), hintf[f].end(), h.hint.begin() + size_t(a) * ns * nr);
        }
        RPA_CHECK(coulomb_apply(g, b.cb, 1, ncol, b.P, b.U, s));
        RPA_CHECK(chi0_apply(cell, g, ncol, b.U, b.D, o, b.xb, h, t, s));
        RPA_CHECK(coulomb_apply(g, b.cb, 1, ncol, b.D, b.R, s));
        for (int a = 0; a < na; ++a) {
            const int f = active[a];
            std::copy(h.hint.begin() + size_t(a) * ns * nr, h.hint.begin() + size_t(a + 1) * ns * nr,
                      hintf[f].begin());
            double* C = b.C + f * sq;
            RPA_HIP(launch_gram(nd, nr, b.P + a * blk, b.R + a * blk, b.part, b.gsplit, C, s));
            RPA_HIP(launch_symmetrize(nr, C, s));
            if (o.sq_order > 0)
                RPA_HIP(launch_sq_energy(nr, C, o.sq_order, weight[f] / (2.0 * M_PI), b.ework,
                                         b.escal + 8 * f, b.info + 8 * f, s));
            else
                RPA_HIP(launch_energy_logdet(nr, C, weight[f] / (2.0 * M_PI), b.ework,
                                             b.escal + 8 * f, b.info + 8 * f, s));
            RPA_HIP(launch_gram(nd, nr, b.R + a * blk, b.R + a * blk, b.part, b.gsplit, b.M + f * sq, s));
            RPA_HIP(launch_chol_inv(nr, b.M + f * sq, b.L + f * sq, b.T + f * sq, b.info + 8 * f + 1, s));
        }
        RPA_HIP(hipMemcpyAsync(escal.data(), b.escal, sizeof(double) * 8 * nfreq,
                               hipMemcpyDeviceToHost, s));
        RPA_HIP(hipMemcpyAsync(info.data(), b.info, sizeof(int) * 8 * nfreq, hipMemcpyDeviceToHost, s));
        RPA_HIP(hipStreamSynchronize(s));
        if (stats) {
            stats->chi0_applies += na;
            stats->subspace_iters_total += na;
        }
        std::vector<int> next;
        for (int a = 0; a < na; ++a) {
            const int f = active[a];
            const double Ef = escal[8 * f];
            if (info[8 * f] != 0 || !std::isfinite(Ef)) {
                if (t.breakdown)
                    return fail(RPA_EBREAKDOWN, "COCG breakdown in " + std::to_string(t.breakdown) +
                                                    " system(s); I - C not positive definite");
                if (t.unconv)
                    return fail(RPA_ENOTPD, std::to_string(t.unconv) + " COCG system(s) hit "
                                            "cocg_max_iter; I - C not positive definite");
                return fail(info[8 * f] != 0 ? RPA_ENOTPD : RPA_EINVAL,
                            info[8 * f] != 0 ? "I - C is not positive definite"
                                             : "non-finite subspace energy");
            }
            if (info[8 * f + 1] != 0)
                return fail(RPA_ENOTPD, "Cholesky of R^T R failed at column " +
                                            std::to_string(info[8 * f + 1]));
            if (Vsave) RPA_HIP(launch_copy(int64_t(blk), b.P + a * blk, Vsave + f * blk, s));
            if (Csave) RPA_HIP(launch_copy(int64_t(sq), b.C + f * sq, Csave + f * sq, s));
            RPA_HIP(launch_gemm_tall_small(nd, nr, b.R + a * blk, b.T + f * sq, b.Vall + f * blk, s));
            E[f] = Ef;
            k[f] += 1;
            bool capped = false;
            const bool stop = subspace_stop(o, k[f], Ef, Eprev[f], &capped);
            Eprev[f] = Ef;
            if (capped) t.subcap += 1;
            if (!stop) next.push_back(f);
        }
        active.swap(next);
    }
    double total = 0.0;
    for (int f = 0; f < nfreq; ++f) {
        total += E[f];
        if (ec_freq) ec_freq[f] = E[f];
        if (iters) iters[f] = k[f];
    }
    *ec = total;
    return RPA_OK;
}


// ------------------------------------------------------------------ multi-cell energy
// Options per cell of a several-cell energy call: without a caller cap the cells, which run
// concurrently, share the default state budget in proportion to the state their blocks
// would need uncapped (all frequencies' systems at once in batched mode).
std::vector<Opts> cell_options(int ncell, const rpa_cell* cells, const int32_t* nr, int nfreq,
                               const Opts& o) {
    std::vector<Opts> out(ncell, o);
    if (ncell < 2 || o.max_systems > 0) return out;
    std::vector<double> full(ncell);
    double sum = 0.0;
    for (int c = 0; c < ncell; ++c) {
        const Grid g = grid_of(&cells[c]);
        const double sys = double(cells[c].n_occ) * nr[c] *
                           (o.freq_mode == RPA_INDEPENDENT ? std::max(1, nfreq) : 1);
        full[c] = sys * double(g.nd()) * state_bytes_per_point(o);
        sum += full[c];
    }
    if (sum <= kStateBudget) return out;
    for (int c = 0; c < ncell; ++c) out[c].state_budget = kStateBudget * full[c] / sum;
    return out;
}

size_t energy_cell_bytes(const Grid& g, int ns, int nr, int nfreq, const Opts& o) {
    Carver dry;
    if (o.freq_mode == RPA_INDEPENDENT) {
        BatchBuf b;
        carve_batch(dry, g, ns, nr, nfreq, o, b);
    } else {
        EnergyBuf b;
        carve_energy(dry, g, ns, nr, o, b);
    }
    return (dry.used + 255) / 256 * 256;
}

// One cell's share of rpa_energy: inputs, its workspace slice, and its results.
struct CellRun {
    const rpa_cell* cell = nullptr;
    int nr = 0;
    const double* V0 = nullptr;
    double* Vsave = nullptr;
    double* Csave = nullptr;
    char* ws = nullptr;
    SolveTally t;
    int applies = 0;
    double ec = 0.0;
    std::vector<double> ecf;
    std::vector<int> its;
    int rc = RPA_OK;
    std::string err;
};

// E_c of one cell on stream s (warm: frequencies in sequence; independent: batched).
int energy_cell(CellRun& r, int nfreq, const double* omega, const double* weight, const Opts& o,
                hipStream_t s) {
    const rpa_cell* cell = r.cell;
    const Grid g = grid_of(cell);
    const int64_t nd = g.nd();
    const int m_r = r.nr;
    rpa_stats st{};
    Carver cv{r.ws, 0};
    int rc = RPA_OK;
    if (o.freq_mode == RPA_INDEPENDENT) {
        BatchBuf b;
        carve_batch(cv, g, cell->n_occ, m_r, nfreq, o, b);
        rc = energy_batched(cell, m_r, nfreq, omega, weight, r.V0, r.Vsave, r.Csave, o, b, r.t,
                            &st, &r.ec, r.ecf.data(), r.its.data(), s);
    } else {
        EnergyBuf b;
        carve_energy(cv, g, cell->n_occ, m_r, o, b);
        rc = coulomb_setup(g, b.sb.cb, s);
        if (rc >= 0) rc = chol_orthonormalize(g, m_r, r.V0, b.Vstart, b.sb, s);
        if (rc >= 0 && hipSuccess != launch_copy(nd * m_r, b.Vstart, b.Vcur, s))
            rc = fail(RPA_EHIP, "copy launch failed");
        double total = 0.0;
        for (int m = 0; m < nfreq && rc >= 0; ++m) {
            double* vs = r.Vsave ? r.Vsave + size_t(m) * nd * m_r : nullptr;
            double* csv = r.Csave ? r.Csave + size_t(m) * m_r * m_r : nullptr;
            SubResult res;
            rc = subspace_iter(cell, g, omega[m], weight[m], m_r, b.Vcur, vs, csv, nullptr, o,
                               b.sb, r.t, &st, res, s, true);
            if (rc < 0) break;
            total += res.E;
            r.ecf[m] = res.E;
            r.its[m] = res.n_iter;
        }
        r.ec = total;
    }
    r.applies = st.chi0_applies;
    r.rc = rc;
    if (rc < 0) r.err = g_last_error;
    return rc;
}

// Several cells at once: one host thread and one stream per cell (default priority), each
// started after the work already queued on the caller's stream, which then waits for all of
// them.  Cells are independent, so the results equal those of the one-cell calls; the GPU is
// shared by the cells' launches instead of running them one after another.
int energy_cells_concurrent(std::vector<CellRun>& run, int nfreq, const double* omega,
                            const double* weight, const std::vector<Opts>& o, hipStream_t s) {
    int dev = 0;
    RPA_HIP(hipGetDevice(&dev));
    hipEvent_t ready;
    RPA_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    RPA_HIP(hipEventRecord(ready, s));
    const int n = int(run.size());
    std::vector<hipStream_t> st(n, nullptr);
    std::vector<hipEvent_t> done(n, nullptr);
    for (int c = 0; c < n; ++c) {
        RPA_HIP(hipStreamCreateWithFlags(&st[c], hipStreamNonBlocking));
        RPA_HIP(hipEventCreateWithFlags(&done[c], hipEventDisableTiming));
        RPA_HIP(hipStreamWaitEvent(st[c], ready, 0));
    }
    std::vector<std::thread> th;
    for (int c = 0; c < n; ++c) {
        th.emplace_back([&, c] {
            if (hipSetDevice(dev) != hipSuccess) {
                run[c].rc = RPA_EHIP;
                run[c].err = "hipSetDevice failed in a cell worker";
                return;
            }
            energy_cell(run[c], nfreq, omega, weight, o[c], st[c]);
            (void)hipEventRecord(done[c], st[c]);
            (void)hipStreamSynchronize(st[c]);
            release_timer();
        });
    }
    for (auto& t : th) t.join();
    int rc = RPA_OK;
    for (int c = 0; c < n; ++c) {
        (void)hipStreamWaitEvent(s, done[c], 0);
        if (run[c].rc < 0 && rc >= 0) {
            rc = run[c].rc;
            set_error("cell " + std::to_string(c) + ": " + run[c].err);
        }
    }
    RPA_HIP(hipStreamSynchronize(s));
    for (int c = 0; c < n; ++c) {
        (void)hipEventDestroy(done[c]);
        (void)hipStreamDestroy(st[c]);
    }
    (void)hipEventDestroy(ready);
    return rc;
}

}  // namespace
}  // namespace rpa

using namespace rpa;

extern "C" {

int rpa_version(void) { return kVersion; }

const char* rpa_error_string(int code) {
    switch (code) {
        case RPA_OK: return "ok";
        case RPA_ENOTCONV: return "COCG did not converge within cocg_max_iter (results written)";
        case RPA_ESUBCAP: return "subspace iteration stopped at subspace_iters before the energy "
                                 "test held (results written)";
        case RPA_EINVAL: return "invalid argument";
        case RPA_EWORKSPACE: return "workspace missing, misaligned or too small";
        case RPA_EBREAKDOWN: return "COCG breakdown";
        case RPA_ENOTPD: return "matrix not positive definite";
        case RPA_EHIP: return "HIP runtime error";
        case RPA_ENOTIMPL: return "not implemented";
        default: return "unknown status";
    }
}

const char* rpa_last_error(void) { return g_last_error.c_str(); }

int rpa_default_options(rpa_options* opt) {
    if (!opt) return fail(RPA_EINVAL, "options pointer is NULL");
    Opts d;
    std::memset(opt, 0, sizeof(*opt));
    opt->precision = d.precision;
    opt->cocg_max_iter = d.cocg_max_iter;
    opt->cocg_tol = d.cocg_tol;
    opt->subspace_iters = d.subspace_iters;
    opt->freq_mode = d.freq_mode;
    opt->ec_tol = d.ec_tol;
    opt->refine_tol = d.refine_tol;
    opt->mixed_min_omega = d.mixed_min_omega;
    opt->max_systems = d.max_systems;
    opt->flags = 0;
    opt->sq_order = d.sq_order;
    opt->cocg_block = 0;
    return RPA_OK;
}

int rpa_workspace_size(int32_t op, int32_t ncell, const rpa_cell* cells, const int32_t* nvec,
                       int32_t nfreq, const rpa_options* opt, size_t* bytes) {
    g_last_error.clear();
    if (!bytes) return fail(RPA_EINVAL, "bytes pointer is NULL");
    if (ncell < 1 || !cells || !nvec) return fail(RPA_EINVAL, "need ncell >= 1, cells and nvec");
    if (op != RPA_OP_ENERGY && ncell != 1) return fail(RPA_EINVAL, "ncell must be 1 for this op");
    Opts o;
    RPA_CHECK(read_opts(opt, &o));
    size_t need = 0;
    std::vector<Opts> copt;   // per-cell options of a several-cell energy call
    for (int c = 0; c < ncell; ++c) {
        RPA_CHECK(check_geometry(&cells[c]));
        if (nvec[c] < 1 || nvec[c] > 65535) return fail(RPA_EINVAL, "nvec must be in [1, 65535]");
        const Grid g = grid_of(&cells[c]);
        const int ns = cells[c].n_occ;
        Carver cv;
        switch (op) {
            case RPA_OP_COULOMB: { CoulombBuf b; carve_coulomb(cv, g, nvec[c], b); break; }
            case RPA_OP_CHI0: {
                RPA_CHECK(check_solver_geometry(&cells[c], o));
                Chi0Buf b; carve_chi0(cv, g, ns, nvec[c], o, false, false, b); break;
            }
            case RPA_OP_SUBSPACE: {
                RPA_CHECK(check_solver_geometry(&cells[c], o));
                SubBuf b; carve_sub(cv, g, ns, nvec[c], o, b); break;
            }
            case RPA_OP_ENERGY: {
                RPA_CHECK(check_solver_geometry(&cells[c], o));
                if (o.freq_mode == RPA_INDEPENDENT && nfreq < 1)
                    return fail(RPA_EINVAL, "nfreq must be >= 1");
                if (copt.empty()) {
                    for (int k = 0; k < ncell; ++k) {
                        RPA_CHECK(check_geometry(&cells[k]));
                        if (nvec[k] < 1 || nvec[k] > 65535)
                            return fail(RPA_EINVAL, "nvec must be in [1, 65535]");
                    }
                    copt = cell_options(ncell, cells, nvec, std::max(1, int(nfreq)), o);
                }
                // cells run concurrently, each in its own slice: the sizes add up
                need += energy_cell_bytes(g, ns, nvec[c], std::max(1, int(nfreq)), copt[c]);
                continue;
            }
            case RPA_OP_BACKWARD: {
                RPA_CHECK(check_solver_geometry(&cells[c], o));
                if (nfreq < 1) return fail(RPA_EINVAL, "nfreq must be >= 1");
                BackBuf b; carve_back(cv, g, ns, nvec[c], o, b); break;
            }
            default: return fail(RPA_EINVAL, "unknown op");
        }
        need = std::max(need, cv.used);
    }
    *bytes = need;
    return RPA_OK;
}

int rpa_apply_coulomb(const rpa_cell* cell, int32_t power, int32_t nvec, const double* in,
                      double* out, void* ws, size_t ws_bytes, void* stream) {
    g_last_error.clear();
    RPA_CHECK(check_geometry(cell));
    if (power != 1 && power != 2) return fail(RPA_EINVAL, "power must be 1 or 2");
    if (nvec < 1 || nvec > 65535) return fail(RPA_EINVAL, "nvec must be in [1, 65535]");
    if (!in || !out) return fail(RPA_EINVAL, "in/out pointer is NULL");
    const Grid g = grid_of(cell);
    Carver dry;
    CoulombBuf b;
    carve_coulomb(dry, g, nvec, b);
    RPA_CHECK(check_ws(ws, ws_bytes, dry.used));
    Carver cv{static_cast<char*>(ws), 0};
    carve_coulomb(cv, g, nvec, b);
    hipStream_t s = static_cast<hipStream_t>(stream);
    RPA_CHECK(coulomb_setup(g, b, s));
    RPA_CHECK(coulomb_apply(g, b, power, nvec, in, out, s));
    return RPA_OK;
}

int rpa_apply_coulomb_noalloc(const rpa_cell* cell, int32_t power, int32_t nvec,
                              const double* in, double* out, void* stream) {
    g_last_error.clear();
    RPA_CHECK(check_geometry(cell));
    if (power != 1 && power != 2) return fail(RPA_EINVAL, "power must be 1 or 2");
    if (nvec < 1 || nvec > 65535) return fail(RPA_EINVAL, "nvec must be in [1, 65535]");
    if (!in || !out) return fail(RPA_EINVAL, "in/out pointer is NULL");
    const Grid g = grid_of(cell);
    const size_t cap = noalloc_scratch_bytes();
    // the 1D bases and one vector's transform buffer must fit; then as many vectors per pass
    // as the scratch holds
    auto need = [&](int k) {
        Carver dry;
        CoulombBuf b;
        carve_coulomb(dry, g, k, b);
        return dry.used;
    };
    if (need(1) > cap)
        return fail(RPA_EWORKSPACE, "grid too large for the static scratch: one vector needs " +
                                        std::to_string(need(1)) + " bytes, the scratch holds " +
                                        std::to_string(cap));
    int chunk = int(std::min<int64_t>(nvec, int64_t((cap - need(1)) / (8 * size_t(g.nd()))) + 1));
    while (chunk > 1 && need(chunk) > cap) --chunk;
    void* base = nullptr;
    RPA_CHECK(noalloc_scratch(&base));
    Carver cv{static_cast<char*>(base), 0};
    CoulombBuf b;
    carve_coulomb(cv, g, chunk, b);
    hipStream_t s = static_cast<hipStream_t>(stream);
    RPA_CHECK(coulomb_setup(g, b, s));
    const int64_t nd = g.nd();
    for (int j0 = 0; j0 < nvec; j0 += chunk) {
        const int nv = std::min(chunk, nvec - j0);
        RPA_CHECK(coulomb_apply(g, b, power, nv, in + nd * j0, out + nd * j0, s));
    }
    return RPA_OK;
}

int rpa_apply_chi0(const rpa_cell* cell, double omega, int32_t nvec, const double* in,
                   double* out, const rpa_options* opt, rpa_stats* stats, void* ws,
                   size_t ws_bytes, void* stream) {
    g_last_error.clear();
    RPA_CHECK(check_cell(cell));
    if (!(omega > 0.0) || !std::isfinite(omega)) return fail(RPA_EINVAL, "omega must be > 0");
    if (nvec < 1 || nvec > 65535) return fail(RPA_EINVAL, "nvec must be in [1, 65535]");
    if (!in || !out) return fail(RPA_EINVAL, "in/out pointer is NULL");
    if (in == out) return fail(RPA_EINVAL, "in and out must not overlap");
    Opts o;
    RPA_CHECK(read_opts(opt, &o));
    RPA_CHECK(check_solver_geometry(cell, o));
    const Grid g = grid_of(cell);
    Carver dry;
    Chi0Buf b;
    carve_chi0(dry, g, cell->n_occ, nvec, o, false, false, b);
    RPA_CHECK(check_ws(ws, ws_bytes, dry.used));
    Carver cv{static_cast<char*>(ws), 0};
    carve_chi0(cv, g, cell->n_occ, nvec, o, false, false, b);
    hipStream_t s = static_cast<hipStream_t>(stream);
    SolveTally t;
    Chi0Host h;
    h.reset(cell->n_occ, nvec, omega);
    RPA_CHECK(chi0_apply(cell, g, nvec, in, out, o, b, h, t, s));
    add_stats(stats, t);
    if (stats) stats->chi0_applies += 1;
    return solve_status(t);
}

int rpa_subspace_iter(const rpa_cell* cell, double omega, double weight, int32_t nr, double* V,
                      double* V_saved, double* C_out, double* ritz_out, double* ec_out,
                      int32_t* n_iter, const rpa_options* opt, rpa_stats* stats, void* ws,
                      size_t ws_bytes, void* stream) {
    g_last_error.clear();
    RPA_CHECK(check_cell(cell));
    if (!(omega > 0.0) || !std::isfinite(omega)) return fail(RPA_EINVAL, "omega must be > 0");
    if (!std::isfinite(weight)) return fail(RPA_EINVAL, "weight must be finite");
    const Grid g = grid_of(cell);
    if (nr < 1 || nr > 4096 || nr > g.nd()) return fail(RPA_EINVAL, "nr must be in [1, min(4096, N_d)]");
    if (!V || !ec_out) return fail(RPA_EINVAL, "V and ec_out are required");
    Opts o;
    RPA_CHECK(read_opts(opt, &o));
    RPA_CHECK(check_solver_geometry(cell, o));
    Carver dry;
    SubBuf b;
    carve_sub(dry, g, cell->n_occ, nr, o, b);
    RPA_CHECK(check_ws(ws, ws_bytes, dry.used));
    Carver cv{static_cast<char*>(ws), 0};
    carve_sub(cv, g, cell->n_occ, nr, o, b);
    hipStream_t s = static_cast<hipStream_t>(stream);
    SolveTally t;
    SubResult res;
    int rc = subspace_iter(cell, g, omega, weight, nr, V, V_saved, C_out, ritz_out, o, b, t, stats,
                           res, s, false);
    add_stats(stats, t);
    if (rc < 0) return rc;
    *ec_out = res.E;
    if (n_iter) *n_iter = res.n_iter;
    return solve_status(t);
}

int rpa_energy(int32_t ncell, const rpa_cell* cells, const int32_t* nr, int32_t nfreq,
               const double* omega, const double* weight, const double* const* V0,
               double* const* Vsave, double* const* Csave, const rpa_options* opt,
               double* ec_out, double* ec_freq_out, int32_t* iters_out, rpa_stats* stats,
               void* ws, size_t ws_bytes, void* stream) {
    g_last_error.clear();
    if (ncell < 1 || !cells || !nr || !V0 || !ec_out)
        return fail(RPA_EINVAL, "need ncell >= 1, cells, nr, V0 and ec_out");
    if (nfreq < 1 || !omega || !weight) return fail(RPA_EINVAL, "need nfreq >= 1, omega, weight");
    for (int m = 0; m < nfreq; ++m) {
        if (!(omega[m] > 0.0) || !std::isfinite(omega[m])) return fail(RPA_EINVAL, "omega must be > 0");
        if (!std::isfinite(weight[m])) return fail(RPA_EINVAL, "weights must be finite");
    }
    Opts o;
    RPA_CHECK(read_opts(opt, &o));
    for (int c = 0; c < ncell; ++c) {
        RPA_CHECK(check_cell(&cells[c]));
        RPA_CHECK(check_solver_geometry(&cells[c], o));
        const Grid g = grid_of(&cells[c]);
        if (nr[c] < 1 || nr[c] > 4096 || nr[c] > g.nd())
            return fail(RPA_EINVAL, "nr must be in [1, min(4096, N_d)]");
        if (!V0[c]) return fail(RPA_EINVAL, "V0 pointer is NULL");
    }
    const std::vector<Opts> copt = cell_options(ncell, cells, nr, nfreq, o);
    // each cell works in its own slice of the workspace (256-byte aligned offsets)
    std::vector<size_t> offs(ncell + 1, 0);
    for (int c = 0; c < ncell; ++c)
        offs[c + 1] = offs[c] + energy_cell_bytes(grid_of(&cells[c]), cells[c].n_occ, nr[c], nfreq,
                                                  copt[c]);
    RPA_CHECK(check_ws(ws, ws_bytes, offs[ncell]));
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<CellRun> run(ncell);
    for (int c = 0; c < ncell; ++c) {
        CellRun& r = run[c];
        r.cell = &cells[c];
        r.nr = nr[c];
        r.V0 = V0[c];
        r.Vsave = (Vsave && Vsave[c]) ? Vsave[c] : nullptr;
        r.Csave = (Csave && Csave[c]) ? Csave[c] : nullptr;
        r.ws = static_cast<char*>(ws) + offs[c];
        r.ecf.assign(nfreq, 0.0);
        r.its.assign(nfreq, 0);
    }
    int rc;
    if (ncell == 1) {
        rc = energy_cell(run[0], nfreq, omega, weight, copt[0], s);
    } else {
        rc = energy_cells_concurrent(run, nfreq, omega, weight, copt, s);
    }
    SolveTally t;
    for (int c = 0; c < ncell; ++c) {
        const CellRun& r = run[c];
        t.iters_total += r.t.iters_total;
        t.systems += r.t.systems;
        t.launches += r.t.launches;
        t.refinements += r.t.refinements;
        t.iters_max = std::max(t.iters_max, r.t.iters_max);
        t.unconv += r.t.unconv;
        t.breakdown += r.t.breakdown;
        t.kernel_ms += r.t.kernel_ms;
        t.point_iters += r.t.point_iters;
        t.fallbacks += r.t.fallbacks;
        t.subcap += r.t.subcap;
        if (stats) {
            stats->chi0_applies += r.applies;
            stats->subspace_iters_total += r.applies;
        }
        ec_out[c] = r.ec;
        for (int m = 0; m < nfreq; ++m) {
            if (ec_freq_out) ec_freq_out[size_t(c) * nfreq + m] = r.ecf[m];
            if (iters_out) iters_out[size_t(c) * nfreq + m] = r.its[m];
        }
    }
    add_stats(stats, t);
    if (rc < 0) return rc;
    return solve_status(t);
}

int rpa_energy_backward(const rpa_cell* cell, int32_t nfreq, const double* omega,
                        const double* weight, int32_t nr, const double* Vsave,
                        const double* Csave, double grad_ec, double* grad_vloc,
                        const rpa_options* opt, rpa_stats* stats, void* ws, size_t ws_bytes,
                        void* stream) {
    g_last_error.clear();
    RPA_CHECK(check_cell(cell));
    if (nfreq < 1 || !omega || !weight) return fail(RPA_EINVAL, "need nfreq >= 1, omega, weight");
    for (int m = 0; m < nfreq; ++m) {
        if (!(omega[m] > 0.0) || !std::isfinite(omega[m])) return fail(RPA_EINVAL, "omega must be > 0");
        if (!std::isfinite(weight[m])) return fail(RPA_EINVAL, "weights must be finite");
    }
    const Grid g = grid_of(cell);
    if (nr < 1 || nr > 4096 || nr > g.nd()) return fail(RPA_EINVAL, "nr must be in [1, min(4096, N_d)]");
    if (!Vsave || !Csave || !grad_vloc) return fail(RPA_EINVAL, "Vsave, Csave, grad_vloc required");
    if (!std::isfinite(grad_ec)) return fail(RPA_EINVAL, "grad_ec must be finite");
    Opts o;
    RPA_CHECK(read_opts(opt, &o));
    RPA_CHECK(check_solver_geometry(cell, o));
    Carver dry;
    BackBuf b;
    carve_back(dry, g, cell->n_occ, nr, o, b);
    RPA_CHECK(check_ws(ws, ws_bytes, dry.used));
    Carver cv{static_cast<char*>(ws), 0};
    carve_back(cv, g, cell->n_occ, nr, o, b);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int ns = cell->n_occ;
    const int64_t nd = g.nd();
    SolveTally t;
    RPA_CHECK(coulomb_setup(g, b.cb, s));
    RPA_HIP(hipMemcpyAsync(b.xb.eps, cell->eps, sizeof(double) * ns, hipMemcpyHostToDevice, s));
    RPA_HIP(launch_fill(nd, 0.0, grad_vloc, s));
    std::vector<double> mu(nr), ck(nr);
    Chi0Host h;
    RPA_CHECK(precond_setup(cell, g, b.xb, h, s));
    for (int m = 0; m < nfreq; ++m) {
        h.reset(ns, nr, omega[m]);
        const double* Vm = Vsave + size_t(m) * nd * nr;
        const double* Cm = Csave + size_t(m) * nr * nr;
        RPA_HIP(launch_syevj(nr, Cm, b.eigwork, b.mu, b.Y, s));
        RPA_HIP(hipMemcpyAsync(mu.data(), b.mu, sizeof(double) * nr, hipMemcpyDeviceToHost, s));
        RPA_HIP(hipStreamSynchronize(s));
        for (int k = 0; k < nr; ++k) ck[k] = weight[m] / (2.0 * M_PI) * (-mu[k] / (1.0 - mu[k]));
        RPA_HIP(hipMemcpyAsync(b.coefk, ck.data(), sizeof(double) * nr, hipMemcpyHostToDevice, s));
        RPA_HIP(launch_gemm_tall_small(nd, nr, Vm, b.Y, b.W, s));
        RPA_CHECK(coulomb_apply(g, b.cb, 1, nr, b.W, b.U, s));
        for (int j0 = 0; j0 < nr; j0 += b.xb.chunk) {
            const int nv = std::min(b.xb.chunk, nr - j0);
            const bool f64 = fp64_in_mixed(b.xb, o, omega[m]);
            RPA_CHECK(solve_chunk(cell, g, o, b.xb, b.U + nd * j0, j0, nv, b.xb.x_complex, h, s,
                                  f64));
            RPA_CHECK(tally(b.xb, ns * nv, nd, t, h, int64_t(j0) * ns, s));
            if (!f64) RPA_CHECK(continue_capped(cell, g, o, b.xb, nv, h, t, s));
            RPA_HIP(launch_grad_accum_d(nd, ns, nv, cell->psi, b.xb.eps, omega[m], b.xb.coeff,
                                        b.xb.dbuf, b.coefk + j0, b.xb.x, false, grad_vloc, s));
        }
        if (stats) stats->chi0_applies += 1;
    }
    RPA_HIP(launch_scale(nd, grad_ec, grad_vloc, s));
    RPA_HIP(hipStreamSynchronize(s));
    add_stats(stats, t);
    return solve_status(t);
}

}  // extern "C"
