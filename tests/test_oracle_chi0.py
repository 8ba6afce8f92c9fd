"""Pins for chi0 by DFPT (Eqs. 7-9) against the sum over states (Eq. 2) and invariants."""
import numpy as np
import pytest

from oracle import chi0, coulomb, fd
from paper_2504_01816_amd import synth


@pytest.fixture(scope="module")
def cell6():
    return synth.small_cell(n=6, h=0.5, n_wells=2, n_occ=3, seed=11)


def test_generator_orbitals_are_eigenpairs_of_oracle_H(cell6):
    c = cell6
    psi = c.psi.T
    R = fd.hamiltonian_apply(psi, c.vloc, c.shape, c.h) - psi * c.eps[None, :]
    assert np.abs(R).max() <= 1e-10 * np.abs(psi).max() * max(1.0, np.abs(c.eps).max())
    np.testing.assert_allclose(psi.T @ psi * c.dV, np.eye(c.n_occ), atol=1e-12)
    # the lowest eigenpairs of the oracle's dense H
    ev = np.linalg.eigvalsh(fd.hamiltonian_dense(c.vloc, c.shape, c.h))
    np.testing.assert_allclose(c.eps, ev[:c.n_occ], atol=1e-11)


@pytest.mark.parametrize("omega", [0.05, 0.7, 5.0])
def test_dfpt_matches_sum_over_states(cell6, omega):
    c = cell6
    U = np.random.default_rng(7).standard_normal((c.nd, 4))
    D, it, st = chi0.chi0_apply(U, c.vloc, c.psi.T, c.eps, omega, c.shape, c.h, 1e-13, 2000)
    X = chi0.chi0_sum_over_states(c.vloc, c.shape, c.h, c.n_occ, omega)
    assert np.abs(X.imag).max() <= 1e-14 * np.abs(X.real).max()
    ref = X.real @ U
    assert np.abs(D - ref).max() <= 1e-10 * np.abs(ref).max()
    assert np.all(st == 0)


def test_projected_rhs_equals_paper_unprojected_form(cell6):
    c = cell6
    U = np.random.default_rng(8).standard_normal((c.nd, 3))
    D, _, _ = chi0.chi0_apply(U, c.vloc, c.psi.T, c.eps, 0.3, c.shape, c.h, 1e-13, 2000)
    Dp = chi0.chi0_apply_unprojected_dense(U, c.vloc, c.psi.T, c.eps, 0.3, c.shape, c.h)
    assert np.abs(D - Dp).max() <= 1e-10 * np.abs(Dp).max()
    # and the dense projected-form matrix agrees too
    M = chi0.chi0_dense_projected(c.vloc, c.psi.T, c.eps, 0.3, c.shape, c.h)
    assert np.abs(M @ U - Dp).max() <= 1e-10 * np.abs(Dp).max()


def test_chi0_symmetric_negative_semidefinite_and_charge_conserving(cell6):
    c = cell6
    X = chi0.chi0_sum_over_states(c.vloc, c.shape, c.h, c.n_occ, 0.4).real
    np.testing.assert_allclose(X, X.T, atol=1e-14 * np.abs(X).max())
    ev = np.linalg.eigvalsh(X)
    assert ev.max() <= 1e-13 * np.abs(ev).max()
    assert np.abs(X @ np.ones(c.nd)).max() <= 1e-12 * np.abs(X).max()
    # eigenvalues of nu^{1/2} chi0 nu^{1/2} are <= 0 (so ln(1 - lambda) is defined)
    N = coulomb.nu_sqrt_dense(c.shape, c.h)
    lam = np.linalg.eigvalsh(N @ X @ N)
    assert lam.max() <= 1e-12 * np.abs(lam).max()


def test_f_sum_rule_large_frequency(cell6):
    # omega^2 u^T chi0(i omega) u -> -sum_n sum_{i != j} (Lap_h)_ij (u_i - u_j)^2 psi_n,i psi_n,j
    c = cell6
    psi = c.psi.T
    u = np.random.default_rng(9).standard_normal(c.nd)
    L = fd.laplacian_dense(c.shape, c.h)
    np.fill_diagonal(L, 0.0)
    diff2 = (u[:, None] - u[None, :]) ** 2
    ref = -sum(np.sum(L * diff2 * np.outer(psi[:, n], psi[:, n])) for n in range(c.n_occ))
    errs = []
    for om in (1e3, 1e4):
        D, _, _ = chi0.chi0_apply(u[:, None], c.vloc, psi, c.eps, om, c.shape, c.h, 1e-14, 200)
        errs.append(abs(om * om * (u @ D[:, 0]) - ref) / abs(ref))
    assert errs[1] < 1e-4
    assert errs[1] < errs[0] / 50.0          # O(omega^-2) approach
