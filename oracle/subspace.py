"""Subspace iteration on nu^{1/2} chi0 nu^{1/2} and the per-frequency energy (oracle).

Algorithm 1, one subspace iteration at frequency omega_m:
    R = N chi0 N V                      (N = nu^{1/2}; chi0 by DFPT)
    C = V^T R                           (projection)
    E_{c,m} from C                      (the paper uses Gauss spectral quadrature on C;
                                         this build takes the exact sum over the Ritz values)
    M = R^T R;  L L^T = M;  V <- R L^{-T}   (Cholesky orthonormalisation)

Energy (Eq. 10): E_{c,m} = (W_m / 2 pi) sum_k g(mu_k) with g(x) = ln(1 - x) + x and
mu the eigenvalues of the symmetrised C = (V^T R + R^T V) / 2 (C is symmetric only up
to the Sternheimer solver error).  Algorithm 1 omits the quadrature weight and the
1/(2 pi); they are applied here per frequency so that the stopping test compares
energies.  E_{c,m} is recomputed from scratch at each subspace iteration.

Stopping (Algorithm 1 loops while |E_{c,m} - E_{c,m}^old| exceeds a threshold): a
fixed iteration count when ec_tol <= 0, otherwise stop at the first k >= 2 with
|E^(k) - E^(k-1)| <= ec_tol |E^(k)|, or at max_iter.
"""
import numpy as np
from scipy.linalg import cholesky, solve_triangular


def g(x):
    """g(x) = ln(1 - x) + x (Eq. 10)."""
    x = np.asarray(x, dtype=np.float64)
    return np.log1p(-x) + x


def g_prime(x):
    """g'(x) = -x / (1 - x)."""
    x = np.asarray(x, dtype=np.float64)
    return -x / (1.0 - x)


def ritz_energy(V, R, weight):
    """(E_{c,m}, mu, C) for one subspace iteration."""
    C = 0.5 * (V.T @ R + R.T @ V)
    mu = np.linalg.eigvalsh(C)
    E = weight / (2.0 * np.pi) * np.sum(g(mu))
    return E, mu, C


def chol_orthonormalize(R):
    """V = R L^{-T} with L L^T = R^T R (lower Cholesky factor)."""
    M = R.T @ R
    L = cholesky(M, lower=True)
    return solve_triangular(L, R.T, lower=True).T


def subspace_iteration(apply_chi0_tilde, V, weight, max_iter, ec_tol=0.0):
    """Run Algorithm 1's inner loop at one frequency.

    apply_chi0_tilde: callable V -> (R, info) with R = nu^{1/2} chi0 nu^{1/2} V.
    V: orthonormal (N_d, N_r) start block.
    Returns dict with E (the reported E_{c,m}), history, mu, C and V_saved (the V that
    produced E), V_next (the block after the last orthonormalisation), n_iter, infos.
    """
    hist, infos = [], []
    E = mu = C = V_saved = None
    k = 0
    while True:
        k += 1
        R, info = apply_chi0_tilde(V)
        infos.append(info)
        E, mu, C = ritz_energy(V, R, weight)
        hist.append(E)
        V_saved = V
        V = chol_orthonormalize(R)
        if ec_tol <= 0.0:
            if k >= max_iter:
                break
        elif k >= max_iter or (k >= 2 and abs(hist[-1] - hist[-2]) <= ec_tol * abs(hist[-1])):
            break
    return dict(E=E, history=np.array(hist), mu=mu, C=C, V_saved=V_saved, V_next=V,
                n_iter=k, infos=infos)
