"""Pins for the oracle's block COCG (the block variant of the COCG solver named in Sec. 3,
with and without the Kronecker shifted-Laplacian preconditioner)."""
import numpy as np
import pytest

from oracle import chi0 as ochi0
from oracle import fd
from oracle.block import blocks_of, bcocg, chi0_apply_block, gauss_solve
from oracle.cocg import NOT_CONVERGED, OK
from oracle.precond import kron_laplacian_inverse, pcocg_batched, precond_shift
from paper_2504_01816_amd import synth


def _sym(rng, n, shift):
    S = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    S = 0.5 * (S + S.T)
    return 2.0 * S / np.linalg.norm(S, 2) + shift * np.eye(n)


def test_gauss_solve_equals_library_solve_and_flags_singular():
    rng = np.random.default_rng(1)
    M = rng.standard_normal((6, 6)) + 1j * rng.standard_normal((6, 6))
    M[0, 0] = 0.0                                   # needs a row swap
    Y = rng.standard_normal((6, 3)) + 1j * rng.standard_normal((6, 3))
    np.testing.assert_allclose(gauss_solve(M, Y), np.linalg.solve(M, Y), rtol=1e-12, atol=1e-12)
    Ms = M.copy()
    Ms[:, 4] = 2.0 * Ms[:, 1]                       # rank deficient
    assert gauss_solve(Ms, Y) is None
    assert gauss_solve(np.zeros((2, 2)), np.ones((2, 2))) is None
    # the breakdown test does not depend on the scale of rows and columns: residual blocks
    # whose columns differ in norm by 1e-10 give rho entries 1e-20 apart
    D = np.diag([1.0, 1e-10, 1.0, 1e-12, 1.0, 1e-9])
    X = gauss_solve(D @ M @ D, D @ Y)
    assert X is not None
    np.testing.assert_allclose(X, np.linalg.solve(D @ M @ D, D @ Y), rtol=1e-10)


def test_block_terminates_within_n_over_k_steps():
    # in exact arithmetic block COCG on k columns spans the whole space after N/k steps (the
    # pure block recurrence: no split, whose threshold would trip on the last, exhausted step)
    rng = np.random.default_rng(2)
    N, k = 24, 4
    A = _sym(rng, N, 3.0 + 0.5j)
    B = rng.standard_normal((N, k)) + 1j * rng.standard_normal((N, k))
    X, it, st = bcocg(lambda P: A @ P, B, 1e-11, 50, split_tol=1e-14)
    assert np.all(st == OK) and it.max() <= N // k
    np.testing.assert_allclose(X, np.linalg.solve(A, B), rtol=1e-10, atol=1e-12)
    # preconditioned by a complex symmetric M (inverse Jacobi): the same bound
    Mi = np.diag(1.0 / np.diag(A))
    X, it, st = bcocg(lambda P: A @ P, B, 1e-11, 50, lambda R: Mi @ R, split_tol=1e-14)
    assert np.all(st == OK) and it.max() <= N // k
    np.testing.assert_allclose(X, np.linalg.solve(A, B), rtol=1e-10, atol=1e-12)


def test_width_one_is_single_vector_pcocg():
    c = synth.small_cell(n=6, h=0.5, n_wells=2, n_occ=3, seed=11)
    rng = np.random.default_rng(3)
    b = rng.standard_normal((c.nd, 1)) + 0j
    shift = c.eps[1] + 0.1j
    applyH = lambda V: fd.hamiltonian_apply(V, c.vloc, c.shape, c.h)
    ks = precond_shift(c.vloc, shift.real) - 1j * shift.imag
    for pre in (False, True):
        mb = (lambda R: kron_laplacian_inverse(R, c.shape, c.h, np.full(R.shape[1], ks))) \
            if pre else None
        mp = (lambda R, idx: kron_laplacian_inverse(R, c.shape, c.h, np.full(len(idx), ks))) \
            if pre else None
        x1, it1, st1 = bcocg(lambda P: applyH(P) - shift * P, b, 1e-11, 500, mb)
        x2, it2, st2 = pcocg_batched(applyH, np.array([shift]), b, 1e-11, 500, mp)
        assert np.array_equal(it1, it2) and np.all(st1 == OK)
        assert np.abs(x1 - x2).max() <= 1e-12 * np.abs(x2).max()


def test_zero_column_never_enters_the_block():
    rng = np.random.default_rng(4)
    A = _sym(rng, 30, 2.5 + 0.3j)
    B = rng.standard_normal((30, 3)) + 1j * rng.standard_normal((30, 3))
    B0 = np.insert(B, 1, 0.0, axis=1)
    X, it, st = bcocg(lambda P: A @ P, B, 1e-10, 100)
    X0, it0, st0 = bcocg(lambda P: A @ P, B0, 1e-10, 100)
    assert it0[1] == 0 and st0[1] == OK and np.all(X0[:, 1] == 0.0)
    assert np.array_equal(np.delete(it0, 1), it)
    assert np.array_equal(np.delete(X0, 1, axis=1), X)


def test_rank_deficient_block_splits_into_single_vector_solves():
    # two equal right-hand sides: P^T A P is singular at the first step, the block splits and
    # every column is solved (the equal pair identically) as by single-vector COCG
    rng = np.random.default_rng(6)
    A = _sym(rng, 40, 1.5 + 0.2j)
    B = rng.standard_normal((40, 3)) + 1j * rng.standard_normal((40, 3))
    B[:, 2] = B[:, 0]
    X, it, st = bcocg(lambda P: A @ P, B, 1e-11, 200)
    assert np.all(st == OK)
    np.testing.assert_allclose(X, np.linalg.solve(A, B), rtol=1e-9, atol=1e-12)
    assert np.array_equal(X[:, 0], X[:, 2]) and it[0] == it[2]
    # after the split (one step along the block directions, then restarts) each column
    # follows single-vector COCG from its own iterate
    _, it1, _ = pcocg_batched(lambda V: A @ V, np.zeros(3), B, 1e-11, 200)
    assert np.all(np.abs(it - it1) <= 2)


def test_deflation_restarts_the_block_on_the_remaining_columns():
    # column 0 is an eigenvector of A, so the first block step solves it exactly and it
    # leaves the block; the other columns then go on as a fresh block solve of their current
    # residuals (beta = 0): the whole run equals one capped step followed by a new solve
    rng = np.random.default_rng(8)
    N = 36
    S = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    S = 0.5 * (S + S.T)
    Qr, _ = np.linalg.qr(rng.standard_normal((N, N)))          # real orthogonal: Q^T Q = I
    lam = 2.0 + 0.3j + rng.uniform(0.0, 1.5, N)
    A = Qr @ np.diag(lam) @ Qr.T + 0.05 * S                      # complex symmetric
    w, V = np.linalg.eig(A)
    B = rng.standard_normal((N, 3)) + 1j * rng.standard_normal((N, 3))
    B[:, 0] = V[:, 0]
    X, it, st = bcocg(lambda P: A @ P, B, 1e-10, 200)
    assert np.all(st == OK) and it[0] == 1
    X1, _, _ = bcocg(lambda P: A @ P, B, 1e-10, 1)
    R1 = B[:, 1:] - A @ X1[:, 1:]
    # block COCG commutes with scaling the columns (B D gives X D), so scaling each residual
    # column to its right-hand side's norm makes one relative tolerance the per-column test
    D = np.linalg.norm(B[:, 1:], axis=0) / np.linalg.norm(R1, axis=0)
    Y, it2, st2 = bcocg(lambda P: A @ P, R1 * D[None, :], 1e-10, 200)
    assert np.all(st2 == OK) and np.all(np.abs(it[1:] - (1 + it2)) <= 1)
    np.testing.assert_allclose(X[:, 1:], X1[:, 1:] + Y / D[None, :], rtol=1e-8, atol=1e-10)


def test_iteration_cap_reports_not_converged():
    rng = np.random.default_rng(5)
    A = _sym(rng, 40, 0.3 + 0.01j)
    B = rng.standard_normal((40, 2)) + 0j
    X, it, st = bcocg(lambda P: A @ P, B, 1e-12, 3)
    assert np.all(it == 3) and np.all(st == NOT_CONVERGED)


def test_blocks_follow_frequency_runs():
    assert blocks_of([1.0] * 6, 4) == [[0, 1, 2, 3], [4, 5]]
    assert blocks_of([2.0, 2.0, 2.0, 0.5, 0.5], 2) == [[0, 1], [2], [3, 4]]
    assert blocks_of([1.0, 2.0, 1.0], 8) == [[0], [1], [2]]


@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
def test_chi0_with_block_solves_equals_plain_dfpt(bc):
    if bc == "periodic":
        c = synth.small_cell(n=8, h=0.5, n_wells=2, n_occ=3, seed=11)
    else:
        c = synth.box_cell((8, 7, 9), 0.5, 2, 3, 21)
    U = np.random.default_rng(7).standard_normal((c.nd, 5))
    for omega in (0.05, 2.0):
        a, it_a, _ = ochi0.chi0_apply(U, c.vloc, c.psi.T, c.eps, omega, c.shape, c.h, 1e-12,
                                      5000, bc=bc)
        for w, pre in ((3, False), (4, True)):
            b, it_b, st = chi0_apply_block(U, c.vloc, c.psi.T, c.eps, omega, c.shape, c.h,
                                           1e-12, 5000, w, precond=pre, bc=bc)
            assert np.all(st == OK)
            assert np.abs(a - b).max() <= 1e-9 * np.abs(a).max()
            assert it_b.sum() < it_a.sum()
