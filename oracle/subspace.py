"""Subspace iteration on nu^{1/2} chi0 nu^{1/2} and the per-frequency energy (oracle).

Algorithm 1, one subspace iteration at frequency omega_m:
    R = N chi0 N V                      (N = nu^{1/2}; chi0 by DFPT)
    C = V^T R                           (projection)
    E_{c,m} from C                      (Gauss spectral quadrature of order N_o on C, as in
                                         Algorithm 1, or, with sq_order = 0, the exact sum
                                         over the Ritz values that SQ converges to)
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


def ritz_energy(V, R, weight, sq_order=0):
    """(E_{c,m}, mu, C) for one subspace iteration; the energy by Gauss SQ of order
    sq_order, or from the Ritz values mu when sq_order = 0."""
    C = 0.5 * (V.T @ R + R.T @ V)
    mu = np.linalg.eigvalsh(C)
    if sq_order > 0:
        E = sq_energy(C, weight, sq_order)
    else:
        E = weight / (2.0 * np.pi) * np.sum(g(mu))
    return E, mu, C


def lanczos_tridiagonal(C, r, n_o):
    """Lanczos on the symmetric matrix C started from the standard basis vector e_r, n_o
    steps (Sec. 3: C ~ L J L^T with L(:, 1) = e_r).  Returns the diagonal a and off-diagonal
    b of the tridiagonal J; stops early (smaller J) when the Krylov space is exhausted."""
    m = C.shape[0]
    q_prev = np.zeros(m)
    q = np.zeros(m)
    q[r] = 1.0
    a, b = [], []
    beta = 0.0
    scale = max(np.abs(C).max(), 1e-300)
    for k in range(n_o):
        w = C @ q - beta * q_prev
        alpha = float(q @ w)
        w = w - alpha * q
        a.append(alpha)
        if k == n_o - 1:
            break
        beta = float(np.linalg.norm(w))
        if beta <= 1e-14 * scale:
            break
        b.append(beta)
        q_prev, q = q, w / beta
    return np.array(a), np.array(b)


def gauss_sq_trace(C, n_o, f):
    """Gauss spectral quadrature of tr f(C) (Sec. 3, Algorithm 1): for every r, the
    eigenvalues (nodes) and squared first eigenvector components (weights) of the Lanczos
    tridiagonal J_r give e_r^T f(C) e_r ~ sum_t Q_r(1, t)^2 f(lambda_t); summed over r."""
    total = 0.0
    for r in range(C.shape[0]):
        a, b = lanczos_tridiagonal(C, r, n_o)
        J = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
        lam, Q = np.linalg.eigh(J)
        total += float(np.sum(Q[0, :] ** 2 * f(lam)))
    return total


def sq_energy(C, weight, n_o):
    """E_{c,m} = W/(2 pi) sum_r sum_t Q_r(1, t)^2 g(lambda_t) (Algorithm 1, SQ method)."""
    return weight / (2.0 * np.pi) * gauss_sq_trace(C, n_o, g)


def chol_orthonormalize(R):
    """V = R L^{-T} with L L^T = R^T R (lower Cholesky factor)."""
    M = R.T @ R
    L = cholesky(M, lower=True)
    return solve_triangular(L, R.T, lower=True).T


def subspace_iteration(apply_chi0_tilde, V, weight, max_iter, ec_tol=0.0, sq_order=0):
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
        E, mu, C = ritz_energy(V, R, weight, sq_order)
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
