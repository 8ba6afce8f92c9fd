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
