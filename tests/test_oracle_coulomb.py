"""Pins for nu and nu^{1/2} (Eq. 5, Kronecker-product scheme of Sec. 3)."""
import numpy as np
import pytest

from oracle import coulomb, fd


@pytest.mark.parametrize("shape,h", [((6, 6, 6), 0.5), ((4, 5, 6), 0.4)])
def test_kronecker_equals_dense_pseudo_inverse_sqrt(shape, h):
    nd = int(np.prod(shape))
    rng = np.random.default_rng(2)
    V = rng.standard_normal((nd, 3))
    dense = coulomb.nu_sqrt_dense(shape, h)
    np.testing.assert_allclose(coulomb.nu_apply(V, shape, h, 1), dense @ V, atol=1e-12)


def test_nu_solves_poisson_on_zero_mean_subspace():
    # -1/(4 pi) Lap_h (nu rho) = rho - mean(rho)   (Eq. 5 with the neutralised density)
    shape, h = (6, 7, 8), 0.45
    nd = int(np.prod(shape))
    rho = np.random.default_rng(3).standard_normal(nd)
    phi = coulomb.nu_apply(rho, shape, h, 2)
    back = -fd.laplacian(phi, shape, h) / (4 * np.pi)
    np.testing.assert_allclose(back, rho - rho.mean(), atol=1e-11)
    assert abs(phi.mean()) < 1e-12


def test_sqrt_squared_is_nu_and_constant_is_null():
    shape, h = (6, 6, 5), 0.5
    nd = int(np.prod(shape))
    rho = np.random.default_rng(4).standard_normal(nd)
    half = coulomb.nu_apply(coulomb.nu_apply(rho, shape, h, 1), shape, h, 1)
    np.testing.assert_allclose(half, coulomb.nu_apply(rho, shape, h, 2), atol=1e-11)
    assert np.abs(coulomb.nu_apply(np.ones(nd), shape, h, 1)).max() < 1e-12


def test_1d_eigenbasis_is_orthonormal_and_matches_symbol():
    for n in (5, 12, 24):
        kap, U = coulomb.eigbasis_1d(n, 0.4)
        np.testing.assert_allclose(U.T @ U, np.eye(n), atol=1e-13)
        np.testing.assert_allclose(-fd.second_diff_dense_1d(n, 0.4) @ U, U * kap, atol=1e-11)
        np.testing.assert_allclose(kap, np.sort(fd.symbol_1d(2 * np.pi * np.arange(n) / n, 0.4)),
                                   atol=1e-11)
        # index 0 is the constant mode
        assert abs(kap[0]) < 1e-12 and np.allclose(np.abs(U[:, 0]), 1 / np.sqrt(n))
