"""Pins for the oracle's COCG solver (Sec. 3)."""
import numpy as np

from oracle.cocg import BREAKDOWN, NOT_CONVERGED, OK, cocg_batched


def _dense_case(n=40, seed=0):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    H = (Q * np.linspace(-1.0, 5.0, n)) @ Q.T
    return H, (lambda V: H @ V)


def test_solves_complex_symmetric_shifted_systems():
    H, applyH = _dense_case()
    n = H.shape[0]
    rng = np.random.default_rng(1)
    shifts = np.array([-2.0 + 0.3j, 0.5 + 1.0j, 1.7 + 0.05j])
    b = rng.standard_normal((n, 3)) + 1j * rng.standard_normal((n, 3))
    x, it, st = cocg_batched(applyH, shifts, b, 1e-12, 500)
    for s in range(3):
        ref = np.linalg.solve(H - shifts[s] * np.eye(n), b[:, s])
        assert np.linalg.norm(x[:, s] - ref) <= 1e-9 * np.linalg.norm(ref)
        r = b[:, s] - (H - shifts[s] * np.eye(n)) @ x[:, s]
        assert np.linalg.norm(r) <= 1e-11 * np.linalg.norm(b[:, s])
    assert np.all(st == OK)
    # harder shifts (closer to the spectrum, smaller imaginary part) need more iterations
    assert it[2] > it[1]


def test_real_spd_case_reduces_to_cg_finite_termination():
    H, applyH = _dense_case(n=12, seed=3)
    # shift below the spectrum: real SPD, COCG = CG, at most n steps in exact arithmetic
    b = np.random.default_rng(2).standard_normal((12, 1)).astype(complex)
    x, it, st = cocg_batched(applyH, np.array([-1.5 + 0j]), b, 1e-10, 100)
    assert it[0] <= 14 and st[0] == OK
    np.testing.assert_allclose(x[:, 0].imag, 0.0, atol=1e-14)


def test_first_step_and_iteration_cap():
    H, applyH = _dense_case(n=20, seed=4)
    b = np.random.default_rng(5).standard_normal((20, 1)) + 0j
    shift = np.array([0.2 + 0.5j])
    x, it, st = cocg_batched(applyH, shift, b, 1e-14, 1)
    A = H - shift[0] * np.eye(20)
    bb = b[:, 0]
    alpha = (bb @ bb) / (bb @ A @ bb)            # unconjugated forms
    np.testing.assert_allclose(x[:, 0], alpha * bb, rtol=1e-13)
    assert it[0] == 1 and st[0] == NOT_CONVERGED


def test_zero_rhs_and_breakdown():
    applyI = lambda V: V
    b = np.zeros((4, 2), dtype=complex)
    b[:, 1] = [1.0, 1j, 0.0, 0.0]                 # b^T b = 0: the bilinear form vanishes
    x, it, st = cocg_batched(applyI, np.array([0.0, 0.0]), b, 1e-10, 50)
    assert it[0] == 0 and st[0] == OK and np.all(x[:, 0] == 0)
    assert st[1] == BREAKDOWN
