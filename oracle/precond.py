"""Kronecker shifted-Laplacian preconditioner and preconditioned COCG (oracle).

Sec. 3 mentions, as an alternative to the projector-based initial guess (whose cost scales
as O(N_r N_s^2 N_d)), a Laplacian-based preconditioner applied through the Kronecker
product formalism, used with the COCG solver.  The preconditioner for the system
(H - eps_n - i omega) x = b is the inverse of the shifted FD Laplacian

    K_s = -1/2 Lap_h + sigma_n - i omega,
    K_s^{-1} = (U_z (x) U_y (x) U_x) diag(1 / (1/2 (kappa_x + kappa_y + kappa_z) + sigma_n - i omega))
               (U_z (x) U_y (x) U_x)^T,

with the 1D eigenbases of Sec. 3's Coulomb construction.  K_s is complex symmetric, so the
preconditioned iteration keeps COCG's unconjugated bilinear form.  The paper does not give
the shift; here sigma_n = max(mean(V_loc) - eps_n, 1/2) Ha, which makes K_s equal to the
system matrix when V_loc is constant (and keeps K_s away from singular otherwise).

Preconditioned COCG from x_0 = 0:

    r_0 = b, z_0 = M r_0, p_0 = z_0, rho_0 = r_0^T z_0
    repeat:  q = A p;  sigma = p^T q;  alpha = rho / sigma
             x <- x + alpha p;  r <- r - alpha q
             stop when ||r||_2 <= tol ||b||_2
             z = M r;  rho' = r^T z;  beta = rho' / rho;  p <- z + beta p

The iteration count is the number of products with A, as for COCG.
"""
import numpy as np

from . import coulomb, fd
from .cocg import BREAKDOWN, NOT_CONVERGED, OK

MIN_SHIFT = 0.5


def precond_shift(vloc, eps_n):
    """sigma_n = max(mean(V_loc) - eps_n, 1/2)."""
    return max(float(np.mean(vloc)) - float(eps_n), MIN_SHIFT)


def kron_laplacian_inverse(R, shape, h, shifts, radius=fd.RADIUS, bc="periodic"):
    """K_s^{-1} R[:, s] for every column s, K_s = -1/2 Lap_h + shifts[s] (complex shift
    sigma - i omega), through the three 1D eigenbases.  R is (N_d, k) complex."""
    n0, n1, n2 = shape
    R = np.asarray(R, dtype=np.complex128)
    vec = R.ndim == 1
    X = R.reshape(n2, n1, n0, -1)
    kx, Ux = coulomb.eigbasis_1d(n0, h, radius, bc)
    ky, Uy = coulomb.eigbasis_1d(n1, h, radius, bc)
    kz, Uz = coulomb.eigbasis_1d(n2, h, radius, bc)
    X = np.einsum('zyxj,xa->zyaj', X, Ux)
    X = np.einsum('zyaj,yb->zbaj', X, Uy)
    X = np.einsum('zbaj,zc->cbaj', X, Uz)
    K = 0.5 * (kz[:, None, None] + ky[None, :, None] + kx[None, None, :])
    X = X / (K[:, :, :, None] + np.asarray(shifts, dtype=np.complex128)[None, None, None, :])
    X = np.einsum('cbaj,zc->zbaj', X, Uz)
    X = np.einsum('zbaj,yb->zyaj', X, Uy)
    X = np.einsum('zyaj,xa->zyxj', X, Ux)
    out = X.reshape(n0 * n1 * n2, -1)
    return out[:, 0] if vec else out


def pcocg_batched(apply_H, shifts, b, tol, max_iter, apply_M=None, breakdown_tol=1e-14):
    """Solve (H - shifts[s]) x_s = b_s for every column s by preconditioned COCG.

    apply_M: callable (R, idx) -> M_s R[:, t] for the columns t of R, which belong to the
    systems idx; None is the identity (plain COCG).  A breakdown (vanishing sigma or rho)
    is reported, not restarted.  Returns (x, iters, status) like cocg_batched.
    """
    b = np.asarray(b, dtype=np.complex128)
    N, S = b.shape
    shifts = np.asarray(shifts, dtype=np.complex128)
    M = (lambda R, idx: R.copy()) if apply_M is None else apply_M

    def nrm(u):
        return np.sqrt(np.sum((u * u.conj()).real, axis=0))

    x = np.zeros_like(b)
    r = b.copy()
    z = M(r, np.arange(S))
    p = z.copy()
    rho = np.sum(r * z, axis=0)
    bnorm = nrm(b)
    iters = np.zeros(S, dtype=np.int64)
    status = np.full(S, OK, dtype=np.int64)
    active = bnorm > 0.0
    while np.any(active):
        idx = np.nonzero(active)[0]
        P = p[:, idx]
        q = apply_H(P) - shifts[None, idx] * P
        sigma = np.sum(P * q, axis=0)
        iters[idx] += 1
        bad = np.abs(sigma) <= breakdown_tol * nrm(P) * nrm(q)
        alpha = np.where(bad, 0.0, rho[idx] / np.where(bad, 1.0, sigma))
        x[:, idx] += alpha[None, :] * P
        r[:, idx] -= alpha[None, :] * q
        conv = (nrm(r[:, idx]) <= tol * bnorm[idx]) & ~bad
        Z = M(r[:, idx], idx)
        rho_new = np.sum(r[:, idx] * Z, axis=0)
        bad = bad | ((np.abs(rho_new) <= breakdown_tol * nrm(r[:, idx]) * nrm(Z)) & ~conv)
        beta = np.where(bad | conv, 0.0, rho_new / np.where(bad | conv, 1.0, rho[idx]))
        p[:, idx] = Z + beta[None, :] * P
        rho[idx] = rho_new
        status[idx[bad]] = BREAKDOWN
        hit_max = (iters[idx] >= max_iter) & ~conv & ~bad
        status[idx[hit_max]] = NOT_CONVERGED
        active[idx[conv | bad | hit_max]] = False
    return x, iters, status


def chi0_apply_precond(U, vloc, psi, eps, omega, shape, h, tol, max_iter, chunk=256,
                       return_solutions=False, bc="periodic"):
    """chi0(i omega) U by DFPT with the Sternheimer systems solved by preconditioned COCG
    (the projected right-hand sides of chi0.build_rhs).  Returns (chi0 U, iters, status[, x])."""
    from .chi0 import build_rhs

    U = np.asarray(U, dtype=np.float64)
    if U.ndim == 1:
        U = U[:, None]
    Nd, Ns = psi.shape
    nvec = U.shape[1]
    bp, _ = build_rhs(U, psi, h ** 3)
    S = Ns * nvec
    eps_s = np.tile(np.asarray(eps, dtype=np.float64), nvec)
    shifts = eps_s + 1j * omega
    sig = np.array([precond_shift(vloc, e) for e in eps_s])
    kshift = sig - 1j * omega                      # K_s = -1/2 Lap_h + sigma - i omega

    def applyH(v):
        return fd.hamiltonian_apply(v, vloc, shape, h, bc=bc)

    iters = np.zeros(S, dtype=np.int64)
    status = np.zeros(S, dtype=np.int64)
    X = np.zeros((Nd, S), dtype=np.complex128) if return_solutions else None
    out = np.zeros((Nd, nvec))
    for s0 in range(0, S, chunk):
        s1 = min(S, s0 + chunk)

        def applyM(R, idx, s0=s0):
            return kron_laplacian_inverse(R, shape, h, kshift[s0 + idx], bc=bc)

        x, it, st = pcocg_batched(applyH, shifts[s0:s1], -bp[:, s0:s1], tol, max_iter, applyM)
        iters[s0:s1] = it
        status[s0:s1] = st
        for t, s in enumerate(range(s0, s1)):
            n, j = s % Ns, s // Ns
            out[:, j] += 4.0 * psi[:, n] * x[:, t].real
        if return_solutions:
            X[:, s0:s1] = x
    if return_solutions:
        return out, iters, status, X
    return out, iters, status
