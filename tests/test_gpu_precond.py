"""GPU parity of the preconditioned COCG path (RPA_FLAG_PRECOND: Kronecker shifted-Laplacian
preconditioner) against the oracle's preconditioned solver and its plain DFPT, element by
element, periodic and isolated, for chi0, the batched-frequency energy and the backward."""
import numpy as np
import pytest
import torch

from oracle import chi0 as ochi0
from oracle import energy as oenergy
from oracle import gradient as ograd
from oracle import precond as opre
from paper_2504_01816_amd import api, synth
from paper_2504_01816_amd import lib as L

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
PRE = L.RPA_FLAG_PRECOND


def say(*a):
    print(*a, flush=True)


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module")
def wl0():
    return synth.workload(0)


@pytest.fixture(scope="module")
def dc0(wl0):
    return api.device_cell(wl0.cells[0], DEV)


@pytest.mark.parametrize("omega", [1.0, 0.02, 8.8])
def test_precond_chi0_matches_oracle(wl0, dc0, omega):
    c = wl0.cells[0]
    say("precond chi0 12^3 omega", omega)
    U = np.random.default_rng(31).standard_normal((6, c.nd))
    out, rc, st = api.rpa_apply_chi0(dc0, omega, torch.tensor(U, device=DEV),
                                     dict(cocg_tol=1e-12, flags=PRE))
    ref, it_ref, st_ref = opre.chi0_apply_precond(U.T, c.vloc, c.psi.T, c.eps, omega, c.shape,
                                                  c.h, 1e-12, 5000)
    plain, it_plain, _ = ochi0.chi0_apply(U.T, c.vloc, c.psi.T, c.eps, omega, c.shape, c.h,
                                          1e-12, 5000)
    say("iterations gpu %d oracle %d plain cocg %d" % (st["cocg_iters_total"], it_ref.sum(),
                                                       it_plain.sum()))
    assert rc == 0 and st["n_unconverged"] == 0 and np.all(st_ref == 0)
    assert rel(out.cpu().numpy().T, ref) < 1e-9
    assert rel(out.cpu().numpy().T, plain) < 1e-9
    # the same recurrence: iteration counts agree to one step per system
    assert abs(st["cocg_iters_total"] - int(it_ref.sum())) <= it_ref.size
    assert st["cocg_iters_total"] < int(it_plain.sum())


def test_precond_chi0_box_matches_oracle():
    c = synth.box_cell((12, 12, 13), 0.5, 2, 4, 21)
    dc = api.device_cell(c, DEV)
    say("precond chi0 isolated box")
    U = np.random.default_rng(32).standard_normal((4, c.nd))
    for omega in (1.0, 0.05):
        out, rc, st = api.rpa_apply_chi0(dc, omega, torch.tensor(U, device=DEV),
                                         dict(cocg_tol=1e-12, flags=PRE))
        ref, it_ref, _ = opre.chi0_apply_precond(U.T, c.vloc, c.psi.T, c.eps, omega, c.shape,
                                                 c.h, 1e-12, 5000, bc="dirichlet")
        assert rc == 0 and rel(out.cpu().numpy().T, ref) < 1e-9
        assert abs(st["cocg_iters_total"] - int(it_ref.sum())) <= it_ref.size


def test_precond_iteration_cap_and_zero_rhs(wl0, dc0):
    c = wl0.cells[0]
    say("precond chi0 cap 3, zero column")
    U = np.random.default_rng(33).standard_normal((3, c.nd))
    U[1] = 0.0
    out, rc, st = api.rpa_apply_chi0(dc0, 0.5, torch.tensor(U, device=DEV),
                                     dict(cocg_max_iter=3, flags=PRE))
    ref, it_ref, st_ref = opre.chi0_apply_precond(U.T, c.vloc, c.psi.T, c.eps, 0.5, c.shape, c.h,
                                                  1e-8, 3)
    assert rc == 1 and st["n_unconverged"] == int((st_ref == 1).sum()) == 8
    assert st["cocg_iters_max"] == 3
    assert float(out[1].abs().max()) == 0.0
    assert rel(out.cpu().numpy().T, ref) < 1e-11


def test_precond_batched_energy_and_backward_match_oracle():
    c = synth.small_cell(n=12, h=0.5, n_wells=2, n_occ=3, seed=11)
    dc = api.device_cell(c, DEV)
    say("precond energy (batched frequencies) + backward")
    om, W = np.array([2.0, 0.3]), np.array([0.6, 0.9])
    V0 = np.random.default_rng(34).standard_normal((6, c.nd))
    o = dict(cocg_tol=1e-12, subspace_iters=2, ec_tol=0.0, freq_mode=L.RPA_INDEPENDENT)
    ref = oenergy.rpa_energy(c.vloc, c.psi.T, c.eps, c.shape, c.h, V0.T, om, W, 1e-12, 5000, 2,
                             mode="independent")
    res = api.rpa_energy(dc, 6, om, W, [torch.tensor(V0, device=DEV)], dict(o, flags=PRE),
                         save=True)
    assert res["status"] == 0
    np.testing.assert_allclose(res["E_freq"][0], ref["E_freq"], rtol=1e-9)
    grad, rc, st = api.rpa_energy_backward(dc, om, W, res["Vsave"][0], res["Csave"][0], 1.0,
                                           dict(o, flags=PRE))
    Vs = [res["Vsave"][0][m].cpu().numpy().T for m in range(2)]
    Cs = [res["Csave"][0][m].cpu().numpy() for m in range(2)]
    gref = ograd.energy_backward(c.vloc, c.psi.T, c.eps, c.shape, c.h, om, W, Vs, Cs, 1e-12, 5000)
    assert rc == 0 and rel(grad.cpu().numpy(), gref) < 1e-8
