"""Pins of the oracle's isolated-box (Dirichlet) path: stencil truncation at the walls,
Coulomb operator without a null space, chi0 by DFPT, and the energy pipeline."""
import numpy as np
import pytest

from oracle import chi0, coulomb, energy, fd, subspace
from paper_2504_01816_amd import synth


def test_second_order_dirichlet_matrix_has_the_sine_spectrum():
    # the radius-1 stencil with zeros beyond the walls is the classic tridiagonal matrix
    # whose eigenvalues are -(4/h^2) sin^2(k pi / (2 (n + 1))): pins the wall truncation
    n, h = 9, 0.3
    D = fd.second_diff_dense_1d(n, h, radius=1, bc="dirichlet")
    k = np.arange(1, n + 1)
    lam = -(4.0 / h ** 2) * np.sin(k * np.pi / (2 * (n + 1))) ** 2
    np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(D)), np.sort(lam), rtol=1e-13)


def test_radius6_dirichlet_matrix_is_the_banded_toeplitz():
    n, h = 15, 0.4
    w = fd.fd_weights()
    D = fd.second_diff_dense_1d(n, h, bc="dirichlet")
    i, j = np.indices((n, n))
    ref = np.where(np.abs(i - j) <= 6, w[np.minimum(np.abs(i - j), 6)], 0.0) / h ** 2
    np.testing.assert_array_equal(D, ref)
    # negative definite (the periodic matrix has the constant in its null space)
    assert np.linalg.eigvalsh(D).max() < 0


def test_stencil_equals_dense_and_interior_accuracy():
    shape, h = (7, 8, 12), 0.45
    rng = np.random.default_rng(3)
    f = rng.standard_normal((np.prod(shape), 2))
    v = rng.standard_normal(np.prod(shape))
    np.testing.assert_allclose(fd.hamiltonian_apply(f, v, shape, h, bc="dirichlet"),
                               fd.hamiltonian_dense(v, shape, h, bc="dirichlet") @ f, atol=1e-12)
    # a Gaussian that vanishes (< 1e-10) within reach of the walls: the truncated stencil
    # equals the periodic one and the 12th-order formula
    n, h = 40, 0.25
    x = (np.arange(n) + 1) * h
    c, s = (n + 1) * h / 2, 0.7
    g1 = np.exp(-(x - c) ** 2 / (2 * s * s))
    d2 = g1 * ((x - c) ** 2 / s ** 4 - 1 / s ** 2)
    G = np.einsum("z,y,x->zyx", g1, g1, g1).reshape(-1)
    lap = (np.einsum("z,y,x->zyx", g1, g1, d2) + np.einsum("z,y,x->zyx", g1, d2, g1)
           + np.einsum("z,y,x->zyx", d2, g1, g1)).reshape(-1)
    got = fd.laplacian(G, (n, n, n), h, bc="dirichlet")
    per = fd.laplacian(G, (n, n, n), h)
    assert np.abs(got - per).max() < 1e-9 * np.abs(lap).max()
    assert np.abs(got - lap).max() < 1e-5 * np.abs(lap).max()


def test_box_coulomb_kronecker_dense_and_poisson():
    shape, h = (7, 8, 12), 0.5
    rng = np.random.default_rng(4)
    f = rng.standard_normal((np.prod(shape), 3))
    N = coulomb.nu_sqrt_dense(shape, h, bc="dirichlet")
    np.testing.assert_allclose(coulomb.nu_apply(f, shape, h, 1, bc="dirichlet"), N @ f,
                               atol=1e-11 * np.abs(N @ f).max())
    phi = coulomb.nu_apply(f, shape, h, 2, bc="dirichlet")        # nu f, no projection
    res = -fd.laplacian(phi, shape, h, bc="dirichlet") / (4 * np.pi) - f
    assert np.abs(res).max() < 1e-10 * np.abs(f).max()
    assert np.linalg.eigvalsh(N).min() > 0


@pytest.fixture(scope="module")
def box7():
    return synth.box_cell((7, 7, 8), 0.5, 2, 3, 31)


def test_box_orbitals_and_dfpt_sum_over_states(box7):
    c = box7
    psi = c.psi.T
    R = fd.hamiltonian_apply(psi, c.vloc, c.shape, c.h, bc="dirichlet") - psi * c.eps[None, :]
    assert np.abs(R).max() < 1e-10 * np.abs(psi).max()
    U = np.random.default_rng(5).standard_normal((c.nd, 3))
    for om in (0.3, 2.0):
        got, _, st = chi0.chi0_apply(U, c.vloc, psi, c.eps, om, c.shape, c.h, 1e-13, 3000,
                                     bc="dirichlet")
        X = chi0.chi0_sum_over_states(c.vloc, c.shape, c.h, c.n_occ, om, bc="dirichlet")
        assert np.abs(got - X @ U).max() < 1e-10 * np.abs(X @ U).max()
        np.testing.assert_allclose(X, X.T, atol=1e-13 * np.abs(X).max())
        assert np.linalg.eigvalsh(X).max() < 1e-13 * np.abs(X).max()
        # a constant potential shift changes no orbital: chi0 1 = 0
        assert np.abs(X @ np.ones(c.nd)).max() < 1e-11 * np.abs(X).max()


def test_box_full_rank_single_iteration_is_the_direct_method(box7):
    c, om = box7, 0.6
    R, _ = energy.chi0_tilde_apply(np.eye(c.nd), c.vloc, c.psi.T, c.eps, om, c.shape, c.h,
                                   1e-13, 3000, bc="dirichlet")
    E, mu, C = subspace.ritz_energy(np.eye(c.nd), R, 1.0)
    N = coulomb.nu_sqrt_dense(c.shape, c.h, bc="dirichlet")
    X = chi0.chi0_sum_over_states(c.vloc, c.shape, c.h, c.n_occ, om, bc="dirichlet")
    lam = np.linalg.eigvalsh(N @ X @ N)
    assert abs(E - np.sum(subspace.g(lam)) / (2 * np.pi)) <= 1e-10 * abs(E)
