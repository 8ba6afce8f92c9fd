"""Derivative of E_c with respect to the grid values of V_loc (oracle).

What is differentiated: E_c = sum_m (W_m / 2 pi) Tr g(C_m) with C_m the symmetrised
projection of nu^{1/2} chi0(i omega_m) nu^{1/2} onto the saved subspace V_m (the one
that produced the reported E_{c,m}); orbitals, eigenvalues and V_m are held fixed and
V_loc enters only through the Sternheimer operators A_n = H - eps_n - i omega.  The
result is the plain partial derivative per grid value (not divided by dV).

Derivation (projected right-hand-side form of chi0, Eqs. 7-9):
  d Tr g(C) = Tr[g'(C) dC] = sum_k g'(mu_k) u_k^T d(chi0) u_k,  C = Y diag(mu) Y^T,
  u_k = nu^{1/2} V Y e_k.
  u^T chi0 u = -4 sum_n Re[b_n^T A_n^{-1} (I - P) b_n],  b_n = psi_n (.) u, P = dV Psi Psi^T,
  and dA_n/dV_r = e_r e_r^T with A_n = A_n^T (complex symmetric), so
  d(u^T chi0 u)/dV_r = 4 sum_n Re[(A_n^{-1} b_n)_r (A_n^{-1}(I - P) b_n)_r].
  With x_n = -A_n^{-1}(I - P) b_n (the forward Sternheimer solution) and, for exact
  eigenpairs, A_n^{-1} P b_n = sum_l psi_l c_l / (eps_l - eps_n - i omega) = -o_n,
  the derivative is 4 sum_n Re[(x_n + o_n)_r (x_n)_r].  The adjoint solve is the
  forward solve (A_n^T = A_n), so nothing beyond the forward systems is needed.
"""
import numpy as np

from . import chi0 as _chi0
from . import coulomb, fd
from .subspace import g_prime


def energy_backward(vloc, psi, eps, shape, h, omegas, weights, V_saved, C_saved,
                    cocg_tol, cocg_max_iter, bc="periodic"):
    """dE_c/dV_loc (N_d,) by the adjoint formula, recomputing the Sternheimer solutions."""
    Nd, Ns = psi.shape
    grad = np.zeros(Nd)
    for m in range(len(omegas)):
        om = float(omegas[m])
        mu, Y = np.linalg.eigh(C_saved[m])
        U = coulomb.nu_apply(V_saved[m] @ Y, shape, h, power=1, bc=bc)
        _, _, _, X, coeff = _chi0.chi0_apply(U, vloc, psi, eps, om, shape, h, cocg_tol,
                                             cocg_max_iter, return_solutions=True, bc=bc)
        nvec = U.shape[1]
        gp = g_prime(mu)
        for s in range(Ns * nvec):
            n, k = s % Ns, s // Ns
            d = coeff[:, s] / (eps - eps[n] - 1j * om)
            o = -(psi @ d)
            x = X[:, s]
            grad += (weights[m] / (2.0 * np.pi)) * gp[k] * 4.0 * ((x + o) * x).real
    return grad


def energy_backward_dense(vloc, psi, eps, shape, h, omegas, weights, V_saved, C_saved,
                          bc="periodic"):
    """Same derivative from dense inverses (tiny grids): 4 sum_n Re[(A^{-1} b)_r (A^{-1}(I-P) b)_r],
    with no use of the eigenpair identity behind o_n."""
    Nd, Ns = psi.shape
    dV = h ** 3
    H = fd.hamiltonian_dense(vloc, shape, h, bc=bc)
    Q = np.eye(Nd) - dV * psi @ psi.T
    grad = np.zeros(Nd)
    for m in range(len(omegas)):
        om = float(omegas[m])
        mu, Y = np.linalg.eigh(C_saved[m])
        U = coulomb.nu_apply(V_saved[m] @ Y, shape, h, power=1, bc=bc)
        gp = g_prime(mu)
        for n in range(Ns):
            Ainv = np.linalg.inv(H - (eps[n] + 1j * om) * np.eye(Nd))
            B = psi[:, n:n + 1] * U                      # (Nd, nvec)
            y1 = Ainv @ B
            y2 = Ainv @ (Q @ B)
            grad += (weights[m] / (2.0 * np.pi)) * 4.0 * ((y1 * y2).real @ gp)
    return grad


def frozen_subspace_energy(vloc, psi, eps, shape, h, omegas, weights, V_saved, cocg_tol,
                           cocg_max_iter):
    """E_c(V_loc) on the fixed saved subspaces: sum_m (W_m/2pi) Tr g(C_m(V_loc)).
    The function whose central finite differences check the adjoint."""
    from .energy import chi0_tilde_apply
    from .subspace import ritz_energy
    E = 0.0
    for m in range(len(omegas)):
        R, _ = chi0_tilde_apply(V_saved[m], vloc, psi, eps, float(omegas[m]), shape, h,
                                cocg_tol, cocg_max_iter)
        E += ritz_energy(V_saved[m], R, float(weights[m]))[0]
    return E
