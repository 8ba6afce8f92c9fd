"""Checks of the seeded input generator against the oracle's own Hamiltonian."""
import numpy as np

from oracle import fd
from paper_2504_01816_amd import synth


def test_wells_and_uniform_cell():
    v = synth.gaussian_wells((10, 10, 10), 0.5, [[1.0, 2.0, 3.0]], [2.0], [1.0])
    assert v.max() <= 0 and -2.01 < v.min() < -1.5
    c = synth.uniform_cell((4, 5, 6), 0.5, 0.25)
    np.testing.assert_allclose(np.sum(c.psi ** 2) * c.dV, 1.0)
    assert c.eps[0] == 0.25


def test_workload0_orbitals_against_oracle_stencil():
    wl = synth.workload(0)
    c = wl.cells[0]
    assert c.shape == (12, 12, 12) and c.n_occ == 4 and wl.n_r == [16]
    psi = c.psi.T
    R = fd.hamiltonian_apply(psi, c.vloc, c.shape, c.h) - psi * c.eps[None, :]
    assert np.abs(R).max() <= 1e-10 * np.abs(psi).max()
    np.testing.assert_allclose(psi.T @ psi * c.dV, np.eye(4), atol=1e-12)
    assert np.all(np.diff(c.eps) > 0) and c.eps_next - c.eps[-1] >= 1e-3
    # the same seed gives the same inputs
    wl2 = synth.workload(0)
    np.testing.assert_array_equal(wl2.V0[0], wl.V0[0])
    np.testing.assert_allclose(wl2.cells[0].vloc, c.vloc, rtol=0, atol=0)


def test_device_ground_state_matches_host():
    # the torch route of the Chebyshev-filtered solver (used to generate the large cells on the
    # GPU) gives the same eigenpairs as the NumPy route, here on the CPU device
    shape, h = (17, 17, 18), 0.45
    rng = np.random.default_rng(4)
    v = synth.gaussian_wells(shape, h, rng.uniform(0, 7, (3, 3)), [2.0, 1.5, 2.5], [1.0, 0.9, 1.1])
    e1, X1, r1 = synth.ground_state(shape, h, v, 5, 3)
    e2, X2, r2 = synth.ground_state(shape, h, v, 5, 3, device="cpu")
    assert r1.max() < 1e-9 and r2.max() < 1e-9
    np.testing.assert_allclose(e2, e1, rtol=0, atol=1e-11)
    np.testing.assert_allclose(np.abs(X2 @ X1.T), np.eye(6), atol=1e-8)


def test_workload_frequency_rule_equals_the_oracle_quadrature():
    # the frequencies and weights every workload feeds to both sides come from synth; they must
    # be the oracle's pinned Gauss-Legendre rule on the map omega = omega0 (1+t)/(1-t), bit for
    # bit, for every size the tests and the bench use (an error in synth's copy would
    # otherwise pass parity, since both sides would integrate with the same wrong nodes)
    from oracle import quadrature
    for n in (1, 2, 3, 8, 16):
        for w0 in (1.0, 0.5):
            om, W = synth.frequency_rule(n, w0)
            om_ref, W_ref = quadrature.frequency_grid(n, w0)
            np.testing.assert_array_equal(om, om_ref)
            np.testing.assert_array_equal(W, W_ref)
    for k in (1, 2, 3, 4):
        wl = synth.workload_frequencies(k)
        om_ref, W_ref = quadrature.frequency_grid(8, 1.0)
        np.testing.assert_array_equal(wl[0], om_ref)
        np.testing.assert_array_equal(wl[1], W_ref)
