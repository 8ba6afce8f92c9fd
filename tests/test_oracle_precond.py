"""Pins for the oracle's Kronecker shifted-Laplacian preconditioner and preconditioned COCG
(the alternative to the projector-based initial guess mentioned in Sec. 3)."""
import numpy as np
import pytest

from oracle import chi0 as ochi0
from oracle import fd
from oracle.cocg import OK, cocg_batched
from oracle.precond import (chi0_apply_precond, kron_laplacian_inverse, pcocg_batched,
                            precond_shift)
from paper_2504_01816_amd import synth


@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
def test_kronecker_inverse_equals_dense_inverse(bc):
    shape, h = (6, 5, 7), 0.45
    nd = 6 * 5 * 7
    L = fd.laplacian_dense(shape, h, bc=bc)
    rng = np.random.default_rng(3)
    R = rng.standard_normal((nd, 3)) + 1j * rng.standard_normal((nd, 3))
    shifts = np.array([0.5 - 1.0j, 2.0 - 0.02j, 0.7 - 30.0j])   # sigma - i omega
    Z = kron_laplacian_inverse(R, shape, h, shifts, bc=bc)
    for s in range(3):
        K = -0.5 * L + shifts[s] * np.eye(nd)
        ref = np.linalg.solve(K, R[:, s])
        assert np.abs(Z[:, s] - ref).max() <= 1e-12 * np.abs(ref).max()


def test_identity_preconditioner_is_plain_cocg():
    c = synth.small_cell(n=6, h=0.5, n_wells=2, n_occ=3, seed=11)
    applyH = lambda V: fd.hamiltonian_apply(V, c.vloc, c.shape, c.h)
    rng = np.random.default_rng(4)
    b = rng.standard_normal((c.nd, 2)) + 0j
    shifts = np.array([c.eps[0] + 0.3j, c.eps[2] + 0.05j])
    x1, it1, st1 = cocg_batched(applyH, shifts, b, 1e-11, 500)
    x2, it2, st2 = pcocg_batched(applyH, shifts, b, 1e-11, 500, apply_M=None)
    assert np.array_equal(it1, it2) and np.all(st2 == OK)
    assert np.abs(x1 - x2).max() <= 1e-13 * np.abs(x1).max()


def test_exact_preconditioner_converges_in_one_step():
    # constant V_loc = 1 and eps = -0.5: sigma = max(1 + 0.5, 1/2) = 1.5, so K_s equals the
    # system matrix H - eps - i omega and one preconditioned step solves the system
    shape, h = (7, 6, 5), 0.5
    nd = 7 * 6 * 5
    vloc = np.full(nd, 1.0)
    eps, omega = -0.5, 0.4
    sig = precond_shift(vloc, eps)
    assert sig == 1.5
    applyH = lambda V: fd.hamiltonian_apply(V, vloc, shape, h)
    applyM = lambda R, idx: kron_laplacian_inverse(R, shape, h, np.full(len(idx), sig - 1j * omega))
    b = np.random.default_rng(5).standard_normal((nd, 1)) + 0j
    x, it, st = pcocg_batched(applyH, np.array([eps + 1j * omega]), b, 1e-12, 50, applyM)
    assert it[0] == 1 and st[0] == OK
    A = fd.hamiltonian_dense(vloc, shape, h) - (eps + 1j * omega) * np.eye(nd)
    np.testing.assert_allclose(x[:, 0], np.linalg.solve(A, b[:, 0]), rtol=1e-11, atol=1e-13)


def test_pcocg_solves_sternheimer_systems_with_fewer_steps():
    c = synth.small_cell(n=8, h=0.5, n_wells=2, n_occ=3, seed=11)
    applyH = lambda V: fd.hamiltonian_apply(V, c.vloc, c.shape, c.h)
    H = fd.hamiltonian_dense(c.vloc, c.shape, c.h)
    rng = np.random.default_rng(6)
    b = rng.standard_normal((c.nd, 3)) + 0j
    shifts = np.array([c.eps[2] + 0.02j, c.eps[0] + 1.0j, c.eps[1] + 20.0j])
    ksh = np.array([precond_shift(c.vloc, s.real) - 1j * s.imag for s in shifts])
    applyM = lambda R, idx: kron_laplacian_inverse(R, c.shape, c.h, ksh[idx])
    x, it, st = pcocg_batched(applyH, shifts, b, 1e-12, 2000, applyM)
    _, it0, _ = cocg_batched(applyH, shifts, b, 1e-12, 2000)
    assert np.all(st == OK)
    for s in range(3):
        ref = np.linalg.solve(H - shifts[s] * np.eye(c.nd), b[:, s])
        assert np.linalg.norm(x[:, s] - ref) <= 1e-9 * np.linalg.norm(ref)
    assert np.all(it < it0)


def test_chi0_with_preconditioned_solves_equals_plain_dfpt():
    c = synth.small_cell(n=8, h=0.5, n_wells=2, n_occ=3, seed=11)
    U = np.random.default_rng(7).standard_normal((c.nd, 3))
    for omega in (0.05, 2.0):
        a, it_a, _ = ochi0.chi0_apply(U, c.vloc, c.psi.T, c.eps, omega, c.shape, c.h, 1e-12, 5000)
        b, it_b, st = chi0_apply_precond(U, c.vloc, c.psi.T, c.eps, omega, c.shape, c.h, 1e-12,
                                         5000)
        assert np.all(st == OK)
        assert np.abs(a - b).max() <= 1e-9 * np.abs(a).max()
        assert it_b.sum() < it_a.sum()
