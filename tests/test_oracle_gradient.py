"""Pins for dE_c/dV_loc (adjoint, projected right-hand-side form): central finite
differences of the frozen-subspace energy and the dense-inverse formula."""
import numpy as np
import pytest

from oracle import energy, gradient, subspace
from paper_2504_01816_amd import synth


@pytest.fixture(scope="module")
def setup():
    c = synth.small_cell(n=6, h=0.5, n_wells=2, n_occ=3, seed=11)
    om, W = np.array([2.0, 0.7]), np.array([0.6, 0.9])
    V0 = np.random.default_rng(6).standard_normal((c.nd, 4))
    res = energy.rpa_energy(c.vloc, c.psi.T, c.eps, c.shape, c.h, V0, om, W, 1e-13, 3000, 3)
    return c, om, W, res


def test_adjoint_matches_central_differences(setup):
    c, om, W, res = setup
    psi = c.psi.T
    G = gradient.energy_backward(c.vloc, psi, c.eps, c.shape, c.h, om, W, res["V_saved"],
                                 res["C_saved"], 1e-13, 3000)
    # the frozen-subspace energy at the base point is the forward E_c
    E0 = gradient.frozen_subspace_energy(c.vloc, psi, c.eps, c.shape, c.h, om, W, res["V_saved"],
                                         1e-13, 3000)
    assert abs(E0 - res["E_c"]) <= 1e-12 * abs(E0)
    pts = np.random.default_rng(2005).choice(c.nd, size=5, replace=False)
    d = 1e-4
    for r in pts:
        e = np.zeros(c.nd)
        e[r] = d
        Ep = gradient.frozen_subspace_energy(c.vloc + e, psi, c.eps, c.shape, c.h, om, W,
                                             res["V_saved"], 1e-13, 3000)
        Em = gradient.frozen_subspace_energy(c.vloc - e, psi, c.eps, c.shape, c.h, om, W,
                                             res["V_saved"], 1e-13, 3000)
        fdg = (Ep - Em) / (2 * d)
        assert abs(fdg - G[r]) <= 1e-6 * np.abs(G).max(), (r, fdg, G[r])


def test_adjoint_matches_dense_formula(setup):
    c, om, W, res = setup
    psi = c.psi.T
    G = gradient.energy_backward(c.vloc, psi, c.eps, c.shape, c.h, om, W, res["V_saved"],
                                 res["C_saved"], 1e-13, 3000)
    Gd = gradient.energy_backward_dense(c.vloc, psi, c.eps, c.shape, c.h, om, W, res["V_saved"],
                                        res["C_saved"])
    assert np.abs(G - Gd).max() <= 1e-9 * np.abs(Gd).max()
    assert np.abs(G).max() > 0
