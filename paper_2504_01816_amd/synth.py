"""Seeded synthetic inputs for the RPA chi0 hot path.

The paper reads Kohn-Sham ground-state orbitals and eigenvalues from files written by
a separate ground-state calculation (Sec. 3) for pseudopotential cells of Si, C and
LiH (Sec. 4).  Those pseudopotentials and geometries are not available here, so every
workload is a synthetic periodic cell with a local potential made of Gaussian wells,

    V_loc(r) = -sum_a D_a sum_{nu in {-1,0,1}^3} exp(-|r - R_a - nu L|^2 / (2 sigma_a^2)),

grid point (x, y, z) at r = h (x, y, z), and a ground state computed here: the lowest
N_s eigenpairs of H = -1/2 Lap_h + V_loc (12th-order periodic finite differences).

This module is the only code the GPU path and the CPU oracle share.  It produces
inputs only: the potential, the orbitals and eigenvalues (as the paper's input files
would), the random start block V0, and random sample points.  It holds none of the
method's arithmetic: the ground-state solver below applies H through its Fourier
symbol (FFT), a different route from the real-space stencils of the oracle and of the
kernels, and the tests check the orbitals against the oracle's own stencil.

Array conventions (column-major blocks, x fastest on the grid):
  vloc  (N_d,)       float64, index x + n0*(y + n1*z)
  psi   (N_s, N_d)   float64, row n = orbital n, grid-normalised (sum psi^2 h^3 = 1)
  eps   (N_s,)       float64, ascending
  V0    (N_r, N_d)   float64, standard normal (row j = trial vector j)
"""
import hashlib
import json
import os
from dataclasses import dataclass, field

import numpy as np
import scipy.fft as sfft
from scipy.linalg import eigh as dense_eigh

FD_RADIUS = 6


@dataclass
class Cell:
    shape: tuple          # (n0, n1, n2)
    h: float
    vloc: np.ndarray      # (N_d,)
    psi: np.ndarray       # (N_s, N_d)
    eps: np.ndarray       # (N_s,)
    eps_next: float       # eigenvalue N_s + 1 (gap check)
    residual: float       # max ||H psi - eps psi|| / ||psi|| from the generator
    seed: int
    meta: dict = field(default_factory=dict)
    bc: str = "periodic"  # or "dirichlet": grid points at (i + 1) h, zero outside the box

    @property
    def nd(self):
        return int(np.prod(self.shape))

    @property
    def n_occ(self):
        return int(self.psi.shape[0])

    @property
    def dV(self):
        return self.h ** 3


@dataclass
class Workload:
    name: str
    cells: list
    n_r: list             # subspace size per cell
    omegas: np.ndarray    # ordered high -> low
    weights: np.ndarray
    cocg_tol: float
    subspace_iters: int
    V0: list              # (N_r, N_d) per cell
    extra: dict = field(default_factory=dict)


# ----------------------------------------------------------------------------- potential

def gaussian_wells(shape, h, centers, depths, sigmas):
    n0, n1, n2 = shape
    L = np.array([n0 * h, n1 * h, n2 * h])
    x = np.arange(n0) * h
    y = np.arange(n1) * h
    z = np.arange(n2) * h
    V = np.zeros((n2, n1, n0))
    for c, D, s in zip(centers, depths, sigmas):
        for ix in (-1, 0, 1):
            ex = np.exp(-(x - c[0] - ix * L[0]) ** 2 / (2 * s * s))
            for iy in (-1, 0, 1):
                ey = np.exp(-(y - c[1] - iy * L[1]) ** 2 / (2 * s * s))
                for iz in (-1, 0, 1):
                    ez = np.exp(-(z - c[2] - iz * L[2]) ** 2 / (2 * s * s))
                    V -= D * ez[:, None, None] * ey[None, :, None] * ex[None, None, :]
    return V.reshape(-1)


def gaussian_wells_box(shape, h, centers, depths, sigmas):
    """Wells in an isolated box (no periodic images); grid point i at (i + 1) h."""
    n0, n1, n2 = shape
    x = (np.arange(n0) + 1) * h
    y = (np.arange(n1) + 1) * h
    z = (np.arange(n2) + 1) * h
    V = np.zeros((n2, n1, n0))
    for c, D, s in zip(centers, depths, sigmas):
        ex = np.exp(-(x - c[0]) ** 2 / (2 * s * s))
        ey = np.exp(-(y - c[1]) ** 2 / (2 * s * s))
        ez = np.exp(-(z - c[2]) ** 2 / (2 * s * s))
        V -= D * ez[:, None, None] * ey[None, :, None] * ex[None, None, :]
    return V.reshape(-1)


# ----------------------------------------------------------------------------- ground state

def _fd_w():
    """Radius-6 centred second-derivative weights w_0 .. w_6 from their closed form."""
    from math import factorial
    M = FD_RADIUS
    w = np.zeros(M + 1)
    for p in range(1, M + 1):
        w[p] = 2.0 * (-1) ** (p + 1) * factorial(M) ** 2 / (p * p * factorial(M - p) * factorial(M + p))
    w[0] = -2.0 * w[1:].sum()
    return w


def _fd_symbol(n, h):
    """Fourier symbol of -D2 for the radius-6 centred formula, from the closed-form weights."""
    M = FD_RADIUS
    w = _fd_w()
    th = 2.0 * np.pi * np.arange(n) / n
    s = -w[0] * np.ones(n)
    for p in range(1, M + 1):
        s -= 2.0 * w[p] * np.cos(p * th)
    return s / (h * h)


class _SpectralH:
    """H = -1/2 Lap_h + V applied through the FFT (Lap_h is circulant on the periodic grid)."""

    def __init__(self, shape, h, vloc, workers=-1):
        n0, n1, n2 = shape
        self.shape = shape
        self.kin = 0.5 * (_fd_symbol(n2, h)[:, None, None] + _fd_symbol(n1, h)[None, :, None]
                          + _fd_symbol(n0, h)[None, None, :])
        self.v = vloc.reshape(n2, n1, n0)
        self.workers = workers

    def __call__(self, X):
        # X: (k, N_d) rows are vectors
        n0, n1, n2 = self.shape
        A = X.reshape(-1, n2, n1, n0)
        F = sfft.fftn(A, axes=(1, 2, 3), workers=self.workers)
        T = sfft.ifftn(F * self.kin[None], axes=(1, 2, 3), workers=self.workers).real
        return (T + self.v[None] * A).reshape(X.shape)

    def upper_bound(self):
        return float(self.kin.max() + self.v.max())

    def dense(self):
        n = int(np.prod(self.shape))
        return self(np.eye(n))


def _rayleigh_ritz(Hop, X):
    Q, _ = np.linalg.qr(X.T)
    Q = Q.T
    HQ = Hop(Q)
    Hs = Q @ HQ.T
    Hs = 0.5 * (Hs + Hs.T)
    ev, W = np.linalg.eigh(Hs)
    return ev, W.T @ Q, W.T @ HQ


def _chebyshev_filter(Hop, X, degree, a, b, a0):
    """Scaled Chebyshev filter damping [a, b] and amplifying below a (a0 ~ lowest eigenvalue)."""
    e = 0.5 * (b - a)
    c = 0.5 * (b + a)
    sigma = e / (a0 - c)
    tau = 2.0 / sigma
    Y = (Hop(X) - c * X) * (sigma / e)
    for _ in range(2, degree + 1):
        s_new = 1.0 / (tau - sigma)
        Ynew = (Hop(Y) - c * Y) * (2.0 * s_new / e) - (sigma * s_new) * X
        X, Y, sigma = Y, Ynew, s_new
    return Y


class _BoxH:
    """H = -1/2 Lap_h + V on an isolated box: the Dirichlet second difference along each axis
    is the banded Toeplitz matrix of the stencil weights (reaches beyond the box read zero),
    applied as a dense n x n matrix per axis."""

    def __init__(self, shape, h, vloc):
        from scipy.linalg import toeplitz
        n0, n1, n2 = shape
        self.shape = shape
        w = _fd_w()

        def T(n):
            col = np.zeros(n)
            col[:min(n, FD_RADIUS + 1)] = w[:min(n, FD_RADIUS + 1)]
            return toeplitz(col) / (h * h)
        self.Tx, self.Ty, self.Tz = T(n0), T(n1), T(n2)
        self.v = vloc.reshape(n2, n1, n0)

    def __call__(self, X):
        n0, n1, n2 = self.shape
        A = X.reshape(-1, n2, n1, n0)
        L = (np.einsum("kzyx,wx->kzyw", A, self.Tx) + np.einsum("kzyx,wy->kzwx", A, self.Ty)
             + np.einsum("kzyx,wz->kwyx", A, self.Tz))
        return (-0.5 * L + self.v[None] * A).reshape(X.shape)

    def upper_bound(self):
        return float(2.0 * sum(np.abs(T).sum(axis=1).max() for T in (self.Tx, self.Ty, self.Tz))
                     + self.v.max())

    def dense(self):
        n = int(np.prod(self.shape))
        return self(np.eye(n))


def box_ground_state(shape, h, vloc, n_states, seed, tol=1e-10, degree=24, max_outer=200):
    """Lowest n_states eigenpairs of H on an isolated box (dense up to 4096 points, else the
    Chebyshev-filtered subspace iteration of ground_state with the box operator)."""
    Hop = _BoxH(shape, h, vloc)
    nd = int(np.prod(shape))
    if nd <= 4096:
        H = Hop.dense()
        H = 0.5 * (H + H.T)
        ev, vec = dense_eigh(H, subset_by_index=[0, n_states - 1])
        X = vec.T
        return ev, X, np.linalg.norm(Hop(X) - ev[:, None] * X, axis=1)
    rng = np.random.default_rng(seed + 7919)
    m = n_states + max(8, n_states // 4)
    X = rng.standard_normal((m, nd))
    ev, X, HX = _rayleigh_ritz(Hop, X)
    b = Hop.upper_bound()
    for _ in range(max_outer):
        X = _chebyshev_filter(Hop, X, degree, ev[-1], b, ev[0])
        ev, X, HX = _rayleigh_ritz(Hop, X)
        res = np.linalg.norm(HX - ev[:, None] * X, axis=1)
        if res[:n_states + 1].max() <= tol:
            break
    return ev[:n_states + 1], X[:n_states + 1], res[:n_states + 1]


def box_cell(shape, h, n_wells, n_occ, seed, tol=1e-10):
    """A seeded isolated cell (Dirichlet boundary): Gaussian wells (D ~ U[1,3], sigma ~
    U[0.8,1.2]) placed at least 3 sigma inside the box, lowest n_occ orbitals occupied; the
    next seed is taken if the occupied/unoccupied gap is below 1e-3 Ha."""
    L = np.array([(n + 1) * h for n in shape])
    for s in range(seed, seed + 50):
        rng = np.random.default_rng(s)
        sig = rng.uniform(0.8, 1.2, n_wells)
        dep = rng.uniform(1.0, 3.0, n_wells)
        cen = 3.0 * sig[:, None] + rng.uniform(0, 1, (n_wells, 3)) * (L[None, :] - 6.0 * sig[:, None])
        vloc = gaussian_wells_box(shape, h, cen, dep, sig)
        ev, X, res = box_ground_state(shape, h, vloc, n_occ + 1, s, tol=tol)
        if ev[n_occ] - ev[n_occ - 1] >= 1e-3:
            psi = X[:n_occ] / np.sqrt(h ** 3)
            idx = np.argmax(np.abs(psi), axis=1)
            psi *= np.sign(psi[np.arange(n_occ), idx])[:, None]
            return Cell(tuple(shape), float(h), vloc, np.ascontiguousarray(psi),
                        ev[:n_occ].copy(), float(ev[n_occ]), float(res[:n_occ].max()), s,
                        dict(seed_requested=seed, seed_used=s, n_wells=n_wells,
                             gap=float(ev[n_occ] - ev[n_occ - 1])), bc="dirichlet")
    raise RuntimeError("no seed with an occupied/unoccupied gap found")


class _SpectralHTorch:
    """_SpectralH on a torch device (input generation only: FFT application of H)."""

    def __init__(self, shape, h, vloc, device):
        import torch
        n0, n1, n2 = shape
        self.shape = shape
        kin = 0.5 * (_fd_symbol(n2, h)[:, None, None] + _fd_symbol(n1, h)[None, :, None]
                     + _fd_symbol(n0, h)[None, None, :])
        self.kin = torch.as_tensor(kin, device=device)
        self.v = torch.as_tensor(vloc.reshape(n2, n1, n0), device=device)
        self.ub = float(kin.max() + vloc.max())

    def __call__(self, X):
        import torch
        n0, n1, n2 = self.shape
        A = X.reshape(-1, n2, n1, n0)
        F = torch.fft.fftn(A, dim=(1, 2, 3))
        T = torch.fft.ifftn(F * self.kin[None], dim=(1, 2, 3)).real
        return (T + self.v[None] * A).reshape(X.shape)

    def upper_bound(self):
        return self.ub


def _ground_state_torch(shape, h, vloc, n_states, seed, tol, degree, max_outer, device):
    """The Chebyshev-filtered subspace iteration of ground_state, run with torch on a device
    (same start block, filter and Rayleigh-Ritz steps; rounding differs from the CPU run)."""
    import torch
    Hop = _SpectralHTorch(shape, h, vloc, device)
    nd = int(np.prod(shape))
    rng = np.random.default_rng(seed + 7919)
    m = n_states + max(8, n_states // 4)
    X = torch.as_tensor(rng.standard_normal((m, nd)), device=device)

    def rr(X):
        Q, _ = torch.linalg.qr(X.T)
        Q = Q.T.contiguous()
        HQ = Hop(Q)
        Hs = Q @ HQ.T
        Hs = 0.5 * (Hs + Hs.T)
        ev, W = torch.linalg.eigh(Hs)
        return ev, W.T @ Q, W.T @ HQ

    def cheb(X, a, b, a0):
        e, c = 0.5 * (b - a), 0.5 * (b + a)
        sigma = e / (a0 - c)
        tau = 2.0 / sigma
        Y = (Hop(X) - c * X) * (sigma / e)
        for _ in range(2, degree + 1):
            s_new = 1.0 / (tau - sigma)
            Ynew = (Hop(Y) - c * Y) * (2.0 * s_new / e) - (sigma * s_new) * X
            X, Y, sigma = Y, Ynew, s_new
        return Y

    ev, X, HX = rr(X)
    b = Hop.upper_bound()
    for _ in range(max_outer):
        X = cheb(X, float(ev[-1]), b, float(ev[0]))
        ev, X, HX = rr(X)
        res = torch.linalg.norm(HX - ev[:, None] * X, dim=1)
        if float(res[:n_states + 1].max()) <= tol:
            break
    k = n_states + 1
    return ev[:k].cpu().numpy(), X[:k].cpu().numpy(), res[:k].cpu().numpy()


def ground_state(shape, h, vloc, n_states, seed, tol=1e-10, degree=24, max_outer=200,
                 device=None):
    """Lowest n_states eigenpairs of H (Euclidean-orthonormal rows), plus residual norms.
    device: a torch device for the iterative solver (None: NumPy/SciPy on the host)."""
    Hop = _SpectralH(shape, h, vloc)
    nd = int(np.prod(shape))
    if nd <= 4096:
        H = Hop.dense()
        H = 0.5 * (H + H.T)
        ev, vec = dense_eigh(H, subset_by_index=[0, n_states - 1])
        X = vec.T
        R = Hop(X) - ev[:, None] * X
        return ev, X, np.linalg.norm(R, axis=1)
    if device is not None:
        return _ground_state_torch(shape, h, vloc, n_states, seed, tol, degree, max_outer, device)
    rng = np.random.default_rng(seed + 7919)
    m = n_states + max(8, n_states // 4)
    X = rng.standard_normal((m, nd))
    ev, X, HX = _rayleigh_ritz(Hop, X)
    b = Hop.upper_bound()
    for _ in range(max_outer):
        X = _chebyshev_filter(Hop, X, degree, ev[-1], b, ev[0])
        ev, X, HX = _rayleigh_ritz(Hop, X)
        res = np.linalg.norm(HX - ev[:, None] * X, axis=1)
        if res[:n_states + 1].max() <= tol:
            break
    return ev[:n_states + 1], X[:n_states + 1], res[:n_states + 1]


def make_cell(shape, h, centers, depths, sigmas, n_occ, seed, gap_min=1e-3, tol=1e-10,
              device=None):
    vloc = gaussian_wells(shape, h, centers, depths, sigmas)
    ev, X, res = ground_state(shape, h, vloc, n_occ + 1, seed, tol=tol, device=device)
    dV = h ** 3
    psi = X[:n_occ] / np.sqrt(dV)
    # deterministic sign: largest-magnitude entry positive
    idx = np.argmax(np.abs(psi), axis=1)
    psi *= np.sign(psi[np.arange(n_occ), idx])[:, None]
    cell = Cell(tuple(shape), float(h), vloc, np.ascontiguousarray(psi), ev[:n_occ].copy(),
                float(ev[n_occ]), float(res[:n_occ].max()), seed)
    cell.meta["gap"] = float(ev[n_occ] - ev[n_occ - 1])
    cell.meta["gap_ok"] = bool(cell.meta["gap"] >= gap_min)
    return cell


def uniform_cell(shape, h, v0=0.0):
    """Constant potential with one occupied orbital: psi_0 = Omega^{-1/2}, eps_0 = v0."""
    nd = int(np.prod(shape))
    omega_vol = nd * h ** 3
    psi = np.full((1, nd), 1.0 / np.sqrt(omega_vol))
    return Cell(tuple(shape), float(h), np.full(nd, float(v0)), psi, np.array([float(v0)]),
                float("nan"), 0.0, 0, meta=dict(uniform=True))


# ----------------------------------------------------------------------------- workloads

def frequency_rule(n=8, omega0=1.0):
    """Gauss-Legendre nodes on [-1, 1] mapped by omega = omega0 (1+t)/(1-t), high -> low."""
    t, w = np.polynomial.legendre.leggauss(n)
    om = omega0 * (1 + t) / (1 - t)
    W = w * 2 * omega0 / (1 - t) ** 2
    o = np.argsort(-om)
    return om[o], W[o]


def random_block(nd, nr, seed):
    return np.random.default_rng(seed).standard_normal((nr, nd))


def _random_wells(rng, n_wells, L, dlo, dhi, slo, shi):
    centers = rng.uniform(0.0, 1.0, size=(n_wells, 3)) * np.asarray(L)[None, :]
    depths = rng.uniform(dlo, dhi, size=n_wells)
    sigmas = rng.uniform(slo, shi, size=n_wells)
    return centers, depths, sigmas


def _cache_path(key):
    d = os.environ.get("RPA_CELL_CACHE")
    if not d:
        return None
    tag = hashlib.sha256(json.dumps(key, sort_keys=True).encode()).hexdigest()[:20]
    return os.path.join(d, "cell_%s.npz" % tag)


def _cell_from_seed(shape, h, n_wells, n_occ, seed, fixed=None, lattice=None, tol=1e-10,
                    device=None):
    """Draw wells from `seed`; if the occupied/unoccupied gap is below 1e-3 Ha, move to the
    next seed (recorded in meta['seed_used']).  With RPA_CELL_CACHE set to a directory, the
    generated cell is stored there (plain arrays, .npz) and reused by later calls with the
    same parameters."""
    key = dict(shape=list(shape), h=h, n_wells=n_wells, n_occ=n_occ, seed=seed,
               fixed=list(fixed) if fixed is not None else None, lattice=lattice, tol=tol,
               solver="host" if device is None else "device")
    path = _cache_path(key)
    if path and os.path.exists(path):
        with np.load(path, allow_pickle=False) as z:
            meta = json.loads(str(z["meta"]))
            return Cell(tuple(int(v) for v in z["shape"]), float(z["h"]), z["vloc"].copy(),
                        z["psi"].copy(), z["eps"].copy(), float(z["eps_next"]),
                        float(z["residual"]), int(z["seed"]), meta)
    cell = _cell_from_seed_compute(shape, h, n_wells, n_occ, seed, fixed, lattice, tol, device)
    if path:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        np.savez(path, shape=np.asarray(cell.shape), h=cell.h, vloc=cell.vloc, psi=cell.psi,
                 eps=cell.eps, eps_next=cell.eps_next, residual=cell.residual, seed=cell.seed,
                 meta=json.dumps(cell.meta))
    return cell


def _cell_from_seed_compute(shape, h, n_wells, n_occ, seed, fixed, lattice, tol, device):
    L = [s * h for s in shape]
    for s in range(seed, seed + 50):
        rng = np.random.default_rng(s)
        if lattice is not None:
            m = lattice
            base = (np.stack(np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij"),
                             -1).reshape(-1, 3) + 0.5) * (np.asarray(L) / m)
            jitter = rng.uniform(-0.1, 0.1, size=base.shape) * (np.asarray(L) / m)
            centers = base + jitter
            depths = rng.uniform(1.0, 3.0, size=len(centers))
            sigmas = rng.uniform(0.8, 1.2, size=len(centers))
        elif fixed is not None:
            centers = rng.uniform(0.0, 1.0, size=(n_wells, 3)) * np.asarray(L)[None, :]
            depths = np.full(n_wells, fixed[0])
            sigmas = np.full(n_wells, fixed[1])
        else:
            centers, depths, sigmas = _random_wells(rng, n_wells, L, 1.0, 3.0, 0.8, 1.2)
        cell = make_cell(shape, h, centers, depths, sigmas, n_occ, s, tol=tol, device=device)
        cell.meta["solver"] = "host" if device is None else "device"
        if cell.meta["gap_ok"]:
            cell.meta.update(seed_requested=seed, seed_used=s, n_wells=len(centers))
            return cell
    raise RuntimeError("no seed with an occupied/unoccupied gap found")


CONFIG_NAMES = {
    0: "cell12_ns4_nr16_w1_fp64",
    1: "cell24_ns16_nr64_gl8",
    2: "cell48_ns64_nr256_gl8",
    3: "six_cells_20to40_gl8",
    4: "cell32_ns32_nr128_gl8_grad",
}


def workload_frequencies(k):
    """(omega, weight) of workload k without generating its cell: the single node omega = 1
    with weight 1 for the 12^3 workload, Gauss-Legendre 8 on the rational map otherwise."""
    if k == 0:
        return np.array([1.0]), np.array([1.0])
    return frequency_rule(8, 1.0)


def workload(k, tol=1e-10, device=None):
    """The five synthetic workloads.  device: torch device for the ground-state solver of
    the larger cells (None: host)."""
    if k == 0:
        c = _cell_from_seed((12, 12, 12), 0.5, 2, 4, 1, fixed=(2.0, 1.0), tol=tol, device=device)
        return Workload(CONFIG_NAMES[0], [c], [16], np.array([1.0]), np.array([1.0]), 1e-10, 5,
                        [random_block(c.nd, 16, 1001)])
    om, W = workload_frequencies(k)
    if k == 1:
        c = _cell_from_seed((24, 24, 24), 0.4, 16, 16, 2, tol=tol, device=device)
        return Workload(CONFIG_NAMES[1], [c], [64], om, W, 1e-8, 0, [random_block(c.nd, 64, 1002)])
    if k == 2:
        c = _cell_from_seed((48, 48, 48), 0.35, 64, 64, 3, lattice=4, tol=tol, device=device)
        return Workload(CONFIG_NAMES[2], [c], [256], om, W, 1e-8, 0, [random_block(c.nd, 256, 1003)])
    if k == 3:
        grids = [20, 24, 28, 32, 36, 40]
        occ = [8, 12, 20, 28, 36, 48]
        cells = [_cell_from_seed((g, g, g), 0.4, o, o, 100 + i, tol=tol, device=device)
                 for i, (g, o) in enumerate(zip(grids, occ))]
        return Workload(CONFIG_NAMES[3], cells, [4 * o for o in occ], om, W, 1e-8, 0,
                        [random_block(c.nd, 4 * c.n_occ, 1100 + i) for i, c in enumerate(cells)])
    if k == 4:
        c = _cell_from_seed((32, 32, 32), 0.4, 24, 32, 5, tol=tol, device=device)
        pts = np.sort(np.random.default_rng(2005).choice(c.nd, size=20, replace=False))
        return Workload(CONFIG_NAMES[4], [c], [128], om, W, 1e-8, 0, [random_block(c.nd, 128, 1005)],
                        extra=dict(fd_points=pts, fd_step=1e-4))
    raise ValueError(k)


def small_cell(n=8, h=0.5, n_wells=2, n_occ=3, seed=11):
    """A tiny random-well cell for unit tests (dense ground state)."""
    return _cell_from_seed((n, n, n), h, n_wells, n_occ, seed)
