"""Pins for the oracle's finite-difference Laplacian and Hamiltonian (Sec. 3, Eq. 4)."""
import os
from fractions import Fraction

import numpy as np

from oracle import fd

GOLD = os.path.join(os.path.dirname(__file__), "golden", "fd_weights_order12.txt")


def test_weights_match_published_table():
    table = {}
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        p, v = line.split()
        table[int(p)] = Fraction(v)
    w = fd.fd_weights_exact(6)
    assert [table[p] for p in range(7)] == w


def test_weights_reproduce_polynomial_second_derivatives():
    # a radius-6 centred formula is exact on x^k for k <= 13: sum_p w_|p| p^k = k(k-1) 0^(k-2)
    w = fd.fd_weights_exact(6)
    for k in range(0, 14):
        s = sum(w[abs(p)] * Fraction(p) ** k for p in range(-6, 7))
        assert s == (2 if k == 2 else 0), k
    # and not on x^14 (order exactly 12)
    assert sum(w[abs(p)] * Fraction(p) ** 14 for p in range(-6, 7)) != 0


def test_plane_wave_eigenvalue_and_continuum_limit():
    n, h = 16, 0.3
    shape = (n, n, n)
    x = np.arange(n)
    for k in (1, 3, 5):
        th = 2 * np.pi * k / n
        # f(x,y,z) = cos(th x) cos(th y) sin(th z) is an eigenfunction with eigenvalue -3 kappa
        F = (np.sin(th * x)[:, None, None] * np.cos(th * x)[None, :, None]
             * np.cos(th * x)[None, None, :]).reshape(-1)
        lap = fd.laplacian(F, shape, h)
        kap = fd.symbol_1d(th, h)
        np.testing.assert_allclose(lap, -3 * kap * F, atol=1e-10 * kap)
    # symbol -> theta^2/h^2 with error O(theta^14)
    th = np.array([5e-2, 1e-1, 2e-1])
    np.testing.assert_allclose(fd.symbol_1d(th, 1.0), th ** 2, rtol=1e-10)
    # a 2nd-order formula would be off by th^2/12 relative: the 12th-order one is far closer
    assert abs(fd.symbol_1d(0.5, 1.0) / 0.25 - 1) < 1e-6


def test_dense_equals_stencil_and_symbol_positive():
    rng = np.random.default_rng(0)
    for shape in [(4, 5, 6), (7, 6, 5)]:
        nd = int(np.prod(shape))
        f = rng.standard_normal(nd)
        L = fd.laplacian_dense(shape, 0.45)
        np.testing.assert_allclose(L @ f, fd.laplacian(f, shape, 0.45), atol=1e-11)
        np.testing.assert_allclose(L, L.T, atol=1e-12)
    th = np.linspace(0, np.pi, 2001)
    s = fd.symbol_1d(th, 1.0)
    assert abs(s[0]) < 1e-13 and np.all(s[1:] > 0) and np.all(np.diff(s) > 0)


def test_small_periodic_grid_wraps_onto_same_point():
    # n = 12: offsets +6 and -6 are the same neighbour and must add (circulant eigenvalues)
    n, h = 12, 0.5
    D = fd.second_diff_dense_1d(n, h)
    kap = np.sort(np.linalg.eigvalsh(-D))
    ref = np.sort(fd.symbol_1d(2 * np.pi * np.arange(n) / n, h))
    np.testing.assert_allclose(kap, ref, atol=1e-12)


def test_hamiltonian_is_symmetric_and_local_potential_diagonal():
    shape, h = (5, 4, 6), 0.5
    nd = int(np.prod(shape))
    rng = np.random.default_rng(1)
    v = rng.standard_normal(nd)
    H = fd.hamiltonian_dense(v, shape, h)
    np.testing.assert_allclose(H, H.T, atol=1e-12)
    f = rng.standard_normal(nd)
    np.testing.assert_allclose(fd.hamiltonian_apply(f, v, shape, h), H @ f, atol=1e-11)
    # the potential enters only on the diagonal
    v2 = rng.standard_normal(nd)
    np.testing.assert_allclose(fd.hamiltonian_dense(v2, shape, h) - H, np.diag(v2 - v), atol=1e-12)
