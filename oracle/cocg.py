"""Conjugate orthogonal conjugate gradient (COCG) for complex-symmetric systems (oracle).

Sec. 3: the Sternheimer systems (H - eps_n - i omega) dpsi = rhs have a complex
symmetric (not Hermitian) matrix, and are solved by COCG, i.e. conjugate
gradients with the unconjugated bilinear form x^T y in place of x^H y
(van der Vorst and Melissen).  Starting from x_0 = 0 (the projected right-hand
side already carries the Galerkin removal of occupied components):

    r_0 = b, p_0 = r_0, rho_0 = r_0^T r_0
    repeat:  q = A p;  sigma = p^T q;  alpha = rho / sigma
             x <- x + alpha p;  r <- r - alpha q
             stop when ||r||_2 <= tol ||b||_2          (Euclidean norm, conjugated)
             rho' = r^T r;  beta = rho' / rho;  p <- r + beta p

The relative-residual stopping rule is the "Sternheimer tolerance" of Sec. 4.1.
The iteration count of a system is the number of products with A.  Breakdown
(a vanishing bilinear form while unconverged) restarts once from the current x
with r = b - A x; a second breakdown is reported.

Vectorised over a batch of independent systems that share the operator up to a
per-system complex shift: A_s = H - shift_s.
"""
import numpy as np

OK, NOT_CONVERGED, BREAKDOWN = 0, 1, 2


def _udot(u, v):
    return np.sum(u * v, axis=0)                  # unconjugated bilinear form


def _nrm(u):
    return np.sqrt(np.sum((u * u.conj()).real, axis=0))


def cocg_batched(apply_H, shifts, b, tol, max_iter, breakdown_tol=1e-14):
    """Solve (H - shifts[s]) x_s = b_s for every column s.

    apply_H: callable mapping an (N, k) complex array to H applied column-wise.
    shifts:  (S,) complex.   b: (N, S) complex right-hand sides.
    Returns (x, iters, status) with x (N, S) complex, iters (S,) int, status (S,) int.
    """
    b = np.asarray(b, dtype=np.complex128)
    N, S = b.shape
    shifts = np.asarray(shifts, dtype=np.complex128)

    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rho = _udot(r, r)
    bnorm = _nrm(b)
    iters = np.zeros(S, dtype=np.int64)
    status = np.zeros(S, dtype=np.int64)
    restarted = np.zeros(S, dtype=bool)
    active = bnorm > 0.0                           # a zero right-hand side gives x = 0
    while np.any(active):
        idx = np.nonzero(active)[0]
        P = p[:, idx]
        q = apply_H(P) - shifts[None, idx] * P
        sigma = _udot(P, q)
        iters[idx] += 1
        bad = np.abs(sigma) <= breakdown_tol * _nrm(P) * _nrm(q)
        alpha = np.where(bad, 0.0, rho[idx] / np.where(bad, 1.0, sigma))
        x[:, idx] += alpha[None, :] * P
        r[:, idx] -= alpha[None, :] * q
        rn = _nrm(r[:, idx])
        conv = (rn <= tol * bnorm[idx]) & ~bad
        rho_new = _udot(r[:, idx], r[:, idx])
        bad = bad | ((np.abs(rho_new) <= breakdown_tol * rn * rn) & ~conv)
        beta = np.where(bad | conv, 0.0, rho_new / np.where(bad | conv, 1.0, rho[idx]))
        p[:, idx] = r[:, idx] + beta[None, :] * P
        rho[idx] = rho_new
        done = conv.copy()
        for t in np.nonzero(bad)[0]:
            s = idx[t]
            if restarted[s]:
                status[s] = BREAKDOWN
                done[t] = True
                continue
            # restart once from the current iterate with the true residual
            restarted[s] = True
            xs = x[:, s:s + 1]
            rs = b[:, s] - (apply_H(xs)[:, 0] - shifts[s] * x[:, s])
            r[:, s] = rs
            p[:, s] = rs
            rho[s] = np.sum(rs * rs)
        hit_max = (iters[idx] >= max_iter) & ~done
        status[idx[hit_max]] = NOT_CONVERGED
        done = done | hit_max
        active[idx[done]] = False
    return x, iters, status
