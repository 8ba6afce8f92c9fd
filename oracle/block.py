"""Block COCG for the Sternheimer systems that share one matrix (oracle).

Sec. 3 names the block variant of the COCG solver, together with the Kronecker Laplacian
preconditioner, as the way to drop the quartic projector-based initial guess.  The systems
(H - eps_n - i omega) x = b_(n,j) of one orbital n and one frequency share their matrix
across the trial vectors j, so a group of them can share one Krylov space: block COCG
(block conjugate gradient with COCG's unconjugated bilinear form, since the matrix and the
preconditioner K_s^{-1} are complex symmetric).  With the k right-hand sides B of a group,
X_0 = 0 and M the preconditioner (the identity for unpreconditioned block COCG):

    R = B, Z = M R, P = Z, rho = R^T Z                                   (k x k)
    repeat:  Q = A P;  alpha = (P^T Q)^{-1} rho
             X <- X + P alpha;  R <- R - Q alpha
             a column stops (is deflated) when ||r_c|| <= tol ||b_c||
             Z = M R;  rho' = R^T Z;  beta = rho^{-1} rho';  P <- Z + P beta;  rho = rho'

Readings (the paper gives no formulas for the block variant): the columns still iterating
form the live set L; a converged column is frozen (its x is final) and every k x k quantity
of the next step is taken on L only (rho and beta on L x L, P and Z on the columns of L),
so the block shrinks as its columns converge; columns with b = 0 are never live.  When L
shrinks, the block restarts on its remaining columns (beta = 0, P_L = Z_L): the directions
kept from the larger block are no longer conjugate within the smaller one, and on the 24^3
cell keeping them leaves single columns at 76-124 steps where their blocks converged in
20-24 (with the restart: 23-24).  The small systems are solved by Gaussian elimination with
partial pivoting after scaling every row, then every column, to a largest modulus of one
(the entries of rho and P^T Q scale with the residual norms of their columns, which differ
by up to the tolerance ratio once some columns near convergence).  A pivot of modulus
<= split_tol = 1e-3 of the scaled matrix means the block has lost rank (its residual columns
have become nearly linearly dependent); the block then splits: each of its live columns
goes on as single-vector (P)COCG from its current x and r.  A failed alpha solve takes that
step with the per-column alpha_c = rho_cc / (p_c^T q_c), and the next direction step
restarts every column with p_c = z_c (beta = 0); a failed beta solve restarts at once.  A
split column with a zero p_c^T q_c or r_c^T z_c breaks down.  (Without the restart on
deflation, a split at 1e-14 left the hardest 24^3 blocks at 76-84 steps and 1e-3 at 26-28;
with the restart no block of that cell splits at either threshold; 1e-2 split blocks that
would converge.)  The iteration count of a column is the number of products with A it took
part in.  Groups are runs of trial vectors with equal frequency, cut into blocks of at most
`width` consecutive vectors from the start of each run.
"""
import numpy as np

from . import fd
from .chi0 import build_rhs
from .cocg import BREAKDOWN, NOT_CONVERGED, OK
from .precond import kron_laplacian_inverse, precond_shift


def gauss_solve(M, Rhs, breakdown_tol=1e-14):
    """M^{-1} Rhs: rows, then columns of M scaled to a largest modulus of one (D_r M D_c),
    Gaussian elimination with partial pivoting (row swaps by largest modulus) on the scaled
    system, x = D_c y; None when a row or column is zero or a pivot's modulus is
    <= breakdown_tol."""
    A = np.array(M, dtype=np.complex128)
    Y = np.array(Rhs, dtype=np.complex128)
    n = A.shape[0]
    rs = np.abs(A).max(axis=1) if n else np.zeros(0)
    if np.any(~(rs > 0.0)):
        return None
    A /= rs[:, None]
    Y /= rs[:, None]
    cs = np.abs(A).max(axis=0)
    if np.any(~(cs > 0.0)):
        return None
    A /= cs[None, :]
    for k in range(n):
        piv = k + int(np.argmax(np.abs(A[k:, k])))
        if not abs(A[piv, k]) > breakdown_tol:
            return None
        if piv != k:
            A[[k, piv]] = A[[piv, k]]
            Y[[k, piv]] = Y[[piv, k]]
        for i in range(k + 1, n):
            f = A[i, k] / A[k, k]
            A[i, k:] -= f * A[k, k:]
            Y[i] -= f * Y[k]
    for k in range(n - 1, -1, -1):
        Y[k] = (Y[k] - A[k, k + 1:] @ Y[k + 1:]) / A[k, k]
    return Y / cs[:, None]


SPLIT_TOL = 1e-3


def bcocg(apply_A, B, tol, max_iter, apply_M=None, split_tol=SPLIT_TOL):
    """Solve A X = B for the k columns of B by (preconditioned) block COCG.

    apply_A, apply_M: callables on (N, k') complex blocks; apply_M None is the identity.
    split_tol: pivot threshold of the scaled small solves below which the block splits.
    Returns (X, iters, status) per column, status OK / NOT_CONVERGED / BREAKDOWN.
    """
    B = np.asarray(B, dtype=np.complex128)
    N, k = B.shape
    M = (lambda R: R.copy()) if apply_M is None else apply_M

    def nrm(u):
        return np.sqrt(np.sum((u * u.conj()).real, axis=0))

    bnorm = nrm(B)
    X = np.zeros_like(B)
    R = B.copy()
    Z = np.zeros_like(B)
    P = np.zeros_like(B)
    iters = np.zeros(k, dtype=np.int64)
    status = np.full(k, OK, dtype=np.int64)
    live = bnorm > 0.0
    rho = np.zeros((k, k), dtype=np.complex128)
    split = 0          # 0: block; 1: split, restart pending; 2: split (single vectors)

    def diag_solve(num, den, cols):
        """num_cc / den_cc per column; a zero denominator breaks the column down."""
        d = np.diag(den).copy()
        bad = d == 0.0
        status[cols[bad]] = BREAKDOWN
        live[cols[bad]] = False
        return np.diag(np.where(bad, 0.0, np.diag(num) / np.where(bad, 1.0, d)))

    L = np.nonzero(live)[0]
    if L.size:
        Z[:, L] = M(R[:, L])
        P[:, L] = Z[:, L]
        rho[np.ix_(L, L)] = R[:, L].T @ Z[:, L]
    while L.size:
        Q = apply_A(P[:, L])
        G = P[:, L].T @ Q
        iters[L] += 1
        alpha = None
        if split == 0:
            alpha = gauss_solve(G, rho[np.ix_(L, L)], split_tol)
            if alpha is None:
                split = 1
        if split:
            alpha = diag_solve(rho[np.ix_(L, L)], G, L)
        X[:, L] += P[:, L] @ alpha
        R[:, L] -= Q @ alpha
        conv = nrm(R[:, L]) <= tol * bnorm[L]
        hit = (iters[L] >= max_iter) & ~conv & live[L]
        status[L[hit]] = NOT_CONVERGED
        live[L[conv | hit]] = False
        shrank = L.size > int(np.count_nonzero(live))
        L = np.nonzero(live)[0]
        if not L.size:
            break
        Z[:, L] = M(R[:, L])
        rho_new = R[:, L].T @ Z[:, L]
        if split == 0 and shrank:
            beta = np.zeros((L.size, L.size), dtype=np.complex128)      # deflated: restart
        elif split == 0:
            beta = gauss_solve(rho[np.ix_(L, L)], rho_new, split_tol)
            if beta is None:
                split = 1
        if split == 1:
            beta = np.zeros((L.size, L.size), dtype=np.complex128)      # restart: p = z
            split = 2
        elif split == 2:
            beta = diag_solve(rho_new, rho[np.ix_(L, L)], L)
        P[:, L] = Z[:, L] + P[:, L] @ beta
        rho[np.ix_(L, L)] = rho_new
        L = np.nonzero(live)[0]
    return X, iters, status


def blocks_of(omega_per_vector, width):
    """Blocks of trial-vector indices: runs of equal frequency, cut into pieces of at most
    `width` consecutive vectors from the start of each run."""
    om = list(omega_per_vector)
    out, j = [], 0
    while j < len(om):
        e = j
        while e < len(om) and om[e] == om[j]:
            e += 1
        for a in range(j, e, width):
            out.append(list(range(a, min(e, a + width))))
        j = e
    return out


def chi0_apply_block(U, vloc, psi, eps, omega, shape, h, tol, max_iter, width, precond=False,
                     return_solutions=False, bc="periodic"):
    """chi0(i omega) U by DFPT with the systems of one orbital solved by block COCG over
    blocks of `width` trial vectors (with the Kronecker shifted-Laplacian preconditioner if
    `precond`).  omega is a scalar or one frequency per column of U; the blocks follow
    blocks_of.  Returns (chi0 U, iters, status[, x]) with systems indexed s = n + N_s j."""
    U = np.asarray(U, dtype=np.float64)
    if U.ndim == 1:
        U = U[:, None]
    Nd, Ns = psi.shape
    nvec = U.shape[1]
    om_v = np.broadcast_to(np.asarray(omega, dtype=np.float64), (nvec,))
    bp, _ = build_rhs(U, psi, h ** 3)
    S = Ns * nvec
    iters = np.zeros(S, dtype=np.int64)
    status = np.zeros(S, dtype=np.int64)
    X = np.zeros((Nd, S), dtype=np.complex128)
    for blk in blocks_of(om_v, width):
        om = float(om_v[blk[0]])
        for n in range(Ns):
            cols = [n + Ns * j for j in blk]
            shift = eps[n] + 1j * om

            def applyA(P, shift=shift):
                return fd.hamiltonian_apply(P, vloc, shape, h, bc=bc) - shift * P

            applyM = None
            if precond:
                ks = precond_shift(vloc, eps[n]) - 1j * om

                def applyM(R, ks=ks):
                    return kron_laplacian_inverse(R, shape, h, np.full(R.shape[1], ks), bc=bc)

            x, it, st = bcocg(applyA, -bp[:, cols], tol, max_iter, applyM)
            X[:, cols] = x
            iters[cols] = it
            status[cols] = st
    out = np.zeros((Nd, nvec))
    for s in range(S):
        n, j = s % Ns, s // Ns
        out[:, j] += 4.0 * psi[:, n] * X[:, s].real
    if return_solutions:
        return out, iters, status, X
    return out, iters, status
