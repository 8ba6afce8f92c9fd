"""Density response chi0(i omega) on the grid (oracle).

Matrix convention: chi0 acts on grid values of a potential perturbation and
returns grid values of the density response, Delta rho = chi0 Delta V (Eq. 7).
Orbitals are grid-normalised (sum_r psi_m psi_n dV = delta_mn, dV = h^3,
trapezoidal rule of Sec. 3), closed shell, N_s doubly occupied.

DFPT form (Eqs. 7-9, Algorithm 1): for every occupied n and trial vector u_j,
    b = psi_n (.) u_j
    c = dV Psi^T b,      b' = b - Psi c        (occupied components removed, Sec. 3)
    (H - eps_n - i omega) x = -b'               (Sternheimer, Eq. 9, solved by COCG)
    (chi0 u_j) = 4 sum_n Re(psi_n (.) x_{n,j})  (Eq. 8)

Removing the occupied components from the right-hand side with x_0 = 0 gives the
same chi0 u as the paper's unprojected right-hand side with a Galerkin initial
guess: the occupied-occupied part of the response is antisymmetric in the
orbital pair and cancels in the sum over n (see chi0_apply_unprojected_dense).

Sum-over-states form (Eq. 2) with all eigenpairs of H, used at tiny sizes:
    chi0(r, r') = 2 dV sum_j sum_k (f_j - f_k) psi_j(r) psi_k(r) psi_k(r') psi_j(r')
                  / (eps_j - eps_k - i omega)
"""
import numpy as np

from . import fd
from .cocg import cocg_batched


def build_rhs(U, psi, dV):
    """Projected right-hand sides for all systems s = n + N_s*j.

    Returns (b_proj, coeff) with b_proj (N_d, N_s*nvec) real and coeff (N_s, N_s*nvec)
    the occupied coefficients c = dV Psi^T (psi_n (.) u_j).
    """
    Nd, Ns = psi.shape
    nvec = U.shape[1]
    b = (psi[:, :, None] * U[:, None, :]).reshape(Nd, Ns * nvec, order='F')
    coeff = dV * (psi.T @ b)
    return b - psi @ coeff, coeff


def chi0_apply(U, vloc, psi, eps, omega, shape, h, tol, max_iter,
               chunk=256, return_solutions=False, bc="periodic"):
    """chi0(i omega) U by DFPT; U is (N_d, nvec) real.  Returns (chi0 U, iters[, x, coeff])."""
    U = np.asarray(U, dtype=np.float64)
    if U.ndim == 1:
        U = U[:, None]
    Nd, Ns = psi.shape
    nvec = U.shape[1]
    dV = h ** 3
    bp, coeff = build_rhs(U, psi, dV)
    S = Ns * nvec
    shifts = np.tile(np.asarray(eps, dtype=np.float64), nvec) + 1j * omega
    iters = np.zeros(S, dtype=np.int64)
    status = np.zeros(S, dtype=np.int64)
    X = np.zeros((Nd, S), dtype=np.complex128) if return_solutions else None
    out = np.zeros((Nd, nvec))

    def applyH(v):
        return fd.hamiltonian_apply(v, vloc, shape, h, bc=bc)

    for s0 in range(0, S, chunk):
        s1 = min(S, s0 + chunk)
        x, it, st = cocg_batched(applyH, shifts[s0:s1], -bp[:, s0:s1], tol, max_iter)
        iters[s0:s1] = it
        status[s0:s1] = st
        for t, s in enumerate(range(s0, s1)):
            n, j = s % Ns, s // Ns
            out[:, j] += 4.0 * psi[:, n] * x[:, t].real
        if return_solutions:
            X[:, s0:s1] = x
    if return_solutions:
        return out, iters, status, X, coeff
    return out, iters, status


def chi0_sum_over_states(vloc, shape, h, n_occ, omega, bc="periodic"):
    """Dense chi0(i omega) from Eq. 2 with every eigenpair of the dense H (tiny grids)."""
    H = fd.hamiltonian_dense(vloc, shape, h, bc=bc)
    dV = h ** 3
    evals, evecs = np.linalg.eigh(H)
    psi = evecs / np.sqrt(dV)                       # grid normalisation
    Nd = H.shape[0]
    f = np.zeros(Nd)
    f[:n_occ] = 1.0
    chi = np.zeros((Nd, Nd), dtype=np.complex128)
    # only pairs with f_j != f_k contribute; loop over the occupied index of the pair
    for a in range(n_occ):
        # j = a occupied, k unoccupied
        k = np.arange(n_occ, Nd)
        phi = psi[:, a:a + 1] * psi[:, k]                         # (Nd, nk)
        w1 = (f[a] - f[k]) / (evals[a] - evals[k] - 1j * omega)   # j = a, k
        w2 = (f[k] - f[a]) / (evals[k] - evals[a] - 1j * omega)   # j = k, k' = a
        chi += (phi * (w1 + w2)[None, :]) @ phi.T
    chi *= 2.0 * dV
    return chi


def chi0_apply_unprojected_dense(U, vloc, psi, eps, omega, shape, h, bc="periodic"):
    """The paper's literal form at tiny size: unprojected right-hand side -psi_n u (Eq. 9),
    solved exactly by a dense complex solve, then Delta rho = 4 sum_n Re(psi_n x_n) (Eq. 8)."""
    U = np.asarray(U, dtype=np.float64)
    if U.ndim == 1:
        U = U[:, None]
    H = fd.hamiltonian_dense(vloc, shape, h, bc=bc)
    Nd, Ns = psi.shape
    out = np.zeros((Nd, U.shape[1]))
    for n in range(Ns):
        A = H - (eps[n] + 1j * omega) * np.eye(Nd)
        x = np.linalg.solve(A, -(psi[:, n:n + 1] * U))
        out += 4.0 * psi[:, n:n + 1] * x.real
    return out


def chi0_dense_projected(vloc, psi, eps, omega, shape, h, bc="periodic"):
    """Dense chi0 of the projected-right-hand-side form, as a function of V_loc with Psi, eps fixed:
        chi0 = -4 sum_n D_n Re[A_n^{-1}] (I - P) D_n,  A_n = H - eps_n - i omega,  P = dV Psi Psi^T.
    At exact eigenpairs this equals the sum-over-states chi0 (tiny grids)."""
    H = fd.hamiltonian_dense(vloc, shape, h, bc=bc)
    Nd, Ns = psi.shape
    dV = h ** 3
    Q = np.eye(Nd) - dV * psi @ psi.T
    chi = np.zeros((Nd, Nd))
    for n in range(Ns):
        Ainv = np.linalg.inv(H - (eps[n] + 1j * omega) * np.eye(Nd))
        D = psi[:, n]
        chi -= 4.0 * D[:, None] * (Ainv.real @ (Q * D[None, :]))
    return chi
