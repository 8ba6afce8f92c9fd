"""GPU: the adjoint gradient dE_c/dV_loc against central finite differences of the same
forward, and the torch.autograd binding.

The gradient holds the orbitals, eigenvalues and each frequency's saved subspace V_m fixed
(the energy differentiated is W_m/2pi sum_k g(mu_k(V_m^T chi0~(V_loc) V_m)), exact for the
reported E_c,m), so the finite difference evaluates exactly that frozen-subspace energy: one
subspace step from V_m, whose reported energy is the Rayleigh-Ritz energy of V_m.
"""
import numpy as np
import pytest
import torch

from paper_2504_01816_amd import api, synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)


def frozen_energy(dc, vloc, om, W, Vm, tol):
    cell = api.DeviceCell(dc.shape, dc.h, vloc, dc.psi, dc.eps, dc.bc)
    r = api.rpa_subspace_iter(cell, om, W, Vm.clone(), dict(cocg_tol=tol, subspace_iters=1,
                                                             ec_tol=0.0), want_ritz=False,
                              want_saved=False)
    return r["E"]


@pytest.fixture(scope="module")
def wl4():
    say("generating the 32^3 gradient workload")
    wl = synth.workload(4, device=DEV)
    return wl, api.device_cell(wl.cells[0], DEV)


@pytest.fixture(scope="module")
def fd_terms(wl4):
    """Per frequency m (computed on first use, kept for the module): the adjoint term of
    dE_c/dV_loc at the 20 seeded points and its central difference (step 1e-4 Ha) of that
    frequency's frozen-subspace energy."""
    wl, dc = wl4
    done = {}

    def term(m):
        if m in done:
            return done[m]
        om, W = wl.omegas[[m]], wl.weights[[m]]
        tol = 1e-12
        say("32^3 forward (3 subspace iterations) at omega %.4g" % om[0])
        res = api.rpa_energy(dc, 128, om, W, [torch.tensor(wl.V0[0], device=DEV)],
                             dict(cocg_tol=tol, subspace_iters=3, ec_tol=0.0), save=True)
        assert res["status"] == 0
        grad, rc, _ = api.rpa_energy_backward(dc, om, W, res["Vsave"][0], res["Csave"][0], 1.0,
                                              dict(cocg_tol=tol))
        assert rc == 0
        pts, dlt = wl.extra["fd_points"], wl.extra["fd_step"]
        g = grad.cpu().numpy()[pts]
        fd = np.zeros(len(pts))
        for i, p in enumerate(pts):
            e = []
            for sgn in (1.0, -1.0):
                v = dc.vloc.clone()
                v[int(p)] += sgn * dlt
                e.append(frozen_energy(dc, v, om[0], W[0], res["Vsave"][0][0], tol))
            fd[i] = (e[0] - e[1]) / (2 * dlt)
        done[m] = (g, fd)
        return done[m]

    return term


@pytest.mark.slow
@pytest.mark.parametrize("m", range(8))
def test_gradient_term_matches_finite_differences_32(fd_terms, m):
    # each frequency's term against the central difference of its frozen-subspace energy: to
    # 1e-5 of the term's largest value, above the difference quotient's noise floor (energies
    # solved to tol 1e-12 carry a few 1e-13 Ha of solver noise, over a step of 2e-4 Ha: a few
    # 1e-9); at the highest frequency the term itself is below 1e-7 and the floor decides
    g, fd = fd_terms(m)
    for gi, fi in zip(g, fd):
        say("adjoint %.10e  fd %.10e" % (gi, fi))
    err = np.abs(g - fd).max()
    say("term %d: max difference %.3e, largest value %.3e" % (m, err, np.abs(fd).max()))
    assert err <= 1e-5 * np.abs(fd).max() + 3e-9


@pytest.mark.slow
def test_gradient_matches_finite_differences_32(fd_terms):
    # dE_c/dV_loc over the whole GL8 rule (the sum of the eight terms) against the central
    # difference of the frozen-subspace E_c at the 20 seeded points: 1e-5 relative
    g = sum(fd_terms(m)[0] for m in range(8))
    fd = sum(fd_terms(m)[1] for m in range(8))
    err = np.abs(g - fd).max() / np.abs(fd).max()
    say("E_c gradient over 8 frequencies: max relative difference %.3e" % err)
    assert err < 1e-5


def test_autograd_binding_matches_backward():
    c = synth.small_cell(n=12, h=0.5, n_wells=2, n_occ=3, seed=11)
    dc = api.device_cell(c, DEV)
    om, W = np.array([2.0, 0.7]), np.array([0.6, 0.9])
    V0 = torch.tensor(np.random.default_rng(6).standard_normal((6, c.nd)), device=DEV)
    opts = dict(cocg_tol=1e-12, subspace_iters=3, ec_tol=0.0)
    v = dc.vloc.clone().requires_grad_(True)
    E = api.RPAEnergy.apply(v, dc, 6, om, W, V0, opts)
    (2.5 * E).backward()
    res = api.rpa_energy(dc, 6, om, W, [V0], opts, save=True)
    assert abs(float(E.detach()) - res["E_c"][0]) <= 1e-14 * abs(res["E_c"][0])
    g, _, _ = api.rpa_energy_backward(dc, om, W, res["Vsave"][0], res["Csave"][0], 2.5, opts)
    assert torch.allclose(v.grad, g, rtol=1e-12, atol=0.0)
