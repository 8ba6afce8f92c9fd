"""GPU parity: the HIP path through the C ABI against the CPU FP64 oracle.

Tolerances: the COCG stopping rule is a relative residual tol; two correct FP64
implementations differ by rounding plus at most one extra COCG step per system, so
chi0 u agrees to a small multiple of tol (relative); energies to 1e-9 relative.
"""
import numpy as np
import pytest
import torch

from oracle import chi0 as ochi0
from oracle import coulomb as ocoul
from oracle import energy as oenergy
from oracle import gradient as ograd
from oracle import subspace as osub
from paper_2504_01816_amd import api, synth
from paper_2504_01816_amd import lib as L

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def wl0():
    return synth.workload(0)


@pytest.fixture(scope="module")
def dc0(wl0):
    return api.device_cell(wl0.cells[0], DEV)


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("shape,h,nvec", [((12, 12, 12), 0.5, 3), ((12, 14, 16), 0.45, 5),
                                          ((24, 24, 24), 0.4, 2)])
def test_coulomb_matches_oracle(shape, h, nvec):
    say("coulomb", shape, h, nvec)
    nd = int(np.prod(shape))
    c = synth.uniform_cell(shape, h)
    dc = api.device_cell(c, DEV)
    X = np.random.default_rng(1).standard_normal((nvec, nd))
    for power in (1, 2):
        out = api.rpa_apply_coulomb(dc, torch.tensor(X, device=DEV), power).cpu().numpy()
        ref = ocoul.nu_apply(X.T, shape, h, power).T
        assert rel(out, ref) < 1e-12, (power, rel(out, ref))


def test_chi0_block_apply_matches_oracle(wl0, dc0):
    c = wl0.cells[0]
    say("chi0 12^3 N_s=4 16 vectors tol 1e-10")
    U = np.random.default_rng(2).standard_normal((16, c.nd))
    out, rc, st = api.rpa_apply_chi0(dc0, 1.0, torch.tensor(U, device=DEV), dict(cocg_tol=1e-10))
    ref, iters, status = ochi0.chi0_apply(U.T, c.vloc, c.psi.T, c.eps, 1.0, c.shape, c.h, 1e-10,
                                          5000)
    assert rc == 0 and st["n_unconverged"] == 0 and st["cocg_systems"] == 64
    assert rel(out.cpu().numpy().T, ref) < 1e-9
    # iteration counts agree to within one step per system
    assert abs(st["cocg_iters_total"] - int(iters.sum())) <= 64
    assert st["cocg_iters_max"] <= iters.max() + 1


@pytest.mark.parametrize("omega", [0.02, 8.8])
def test_chi0_low_and_high_frequency(wl0, dc0, omega):
    c = wl0.cells[0]
    say("chi0 omega", omega)
    U = np.random.default_rng(3).standard_normal((4, c.nd))
    out, rc, st = api.rpa_apply_chi0(dc0, omega, torch.tensor(U, device=DEV), dict(cocg_tol=1e-10))
    ref, _, _ = ochi0.chi0_apply(U.T, c.vloc, c.psi.T, c.eps, omega, c.shape, c.h, 1e-10, 5000)
    assert rc == 0 and rel(out.cpu().numpy().T, ref) < 1e-9


def test_chi0_chunking_determinism_and_zero_rhs(wl0, dc0):
    c = wl0.cells[0]
    say("chi0 chunking / determinism / zero column")
    U = np.random.default_rng(4).standard_normal((6, c.nd))
    U[2] = 0.0                                          # a zero trial vector
    X = torch.tensor(U, device=DEV)
    a, rc, st = api.rpa_apply_chi0(dc0, 0.7, X)
    b, _, _ = api.rpa_apply_chi0(dc0, 0.7, X)
    assert torch.equal(a, b)                            # bitwise reproducible
    assert rc == 0 and float(a[2].abs().max()) == 0.0
    ch, rc2, st2 = api.rpa_apply_chi0(dc0, 0.7, X, dict(max_systems=8))  # chunks of 2 vectors
    assert rc2 == 0 and rel(ch.cpu().numpy(), a.cpu().numpy()) < 1e-12
    assert st2["cocg_systems"] == 24


def test_chi0_iteration_cap_reports_not_converged(wl0, dc0):
    c = wl0.cells[0]
    say("chi0 max_iter=2")
    U = np.random.default_rng(5).standard_normal((2, c.nd))
    out, rc, st = api.rpa_apply_chi0(dc0, 1.0, torch.tensor(U, device=DEV), dict(cocg_max_iter=2))
    assert rc == 1 and st["n_unconverged"] == 8 and st["cocg_iters_max"] == 2
    # two COCG steps of the oracle give the same partial result
    ref, _, _ = ochi0.chi0_apply(U.T, c.vloc, c.psi.T, c.eps, 1.0, c.shape, c.h, 1e-8, 2)
    assert rel(out.cpu().numpy().T, ref) < 1e-11


@pytest.fixture(scope="module")
def oracle_e0(wl0):
    c = wl0.cells[0]
    return oenergy.rpa_energy(c.vloc, c.psi.T, c.eps, c.shape, c.h, wl0.V0[0].T, wl0.omegas,
                              wl0.weights, 1e-10, 5000, 5)


def test_energy_workload0_matches_oracle(wl0, dc0, oracle_e0):
    say("rpa_energy 12^3 N_r=16 5 iterations")
    V0 = torch.tensor(wl0.V0[0], device=DEV)
    res = api.rpa_energy(dc0, 16, wl0.omegas, wl0.weights, [V0],
                         dict(cocg_tol=1e-10, subspace_iters=5, ec_tol=0.0), save=True)
    E = res["E_c"][0]
    say("E_c gpu %.15e oracle %.15e" % (E, oracle_e0["E_c"]))
    assert res["status"] == 0 and res["iters"][0, 0] == 5
    assert abs(E - oracle_e0["E_c"]) <= 1e-9 * abs(oracle_e0["E_c"])
    # saved subspace and C reproduce the reported energy
    C = res["Csave"][0][0].cpu().numpy()
    mu = np.linalg.eigvalsh(0.5 * (C + C.T))
    assert abs(np.sum(osub.g(mu)) / (2 * np.pi) - E) <= 1e-12 * abs(E)
    np.testing.assert_allclose(np.sort(mu), np.sort(oracle_e0["mu"][0]), rtol=1e-8, atol=1e-12)


def test_subspace_iter_ritz_values(wl0, dc0, oracle_e0):
    say("rpa_subspace_iter ritz")
    from oracle.subspace import chol_orthonormalize
    V = torch.tensor(chol_orthonormalize(wl0.V0[0].T).T.copy(), device=DEV)
    r = api.rpa_subspace_iter(dc0, 1.0, 1.0, V, dict(cocg_tol=1e-10, subspace_iters=5, ec_tol=0.0))
    assert r["n_iter"] == 5
    assert abs(r["E"] - oracle_e0["E_c"]) <= 1e-9 * abs(oracle_e0["E_c"])
    np.testing.assert_allclose(r["ritz"], np.sort(oracle_e0["mu"][0]), rtol=1e-8, atol=1e-12)
    # returned V is orthonormal
    Vn = V.cpu().numpy()
    assert np.abs(Vn @ Vn.T - np.eye(16)).max() < 1e-10


def test_uniform_potential_closed_form_16():
    say("uniform potential 16^3 first shell")
    shape, h, om = (16, 16, 16), 0.5, 1.0
    c = synth.uniform_cell(shape, h, 0.0)
    dc = api.device_cell(c, DEV)
    from oracle import fd
    kap = (fd.symbol_1d(2 * np.pi * np.arange(16) / 16, h)[:, None, None]
           + fd.symbol_1d(2 * np.pi * np.arange(16) / 16, h)[None, :, None]
           + fd.symbol_1d(2 * np.pi * np.arange(16) / 16, h)[None, None, :]).reshape(-1)
    lam = -(8 * np.pi / (c.nd * h ** 3)) / (kap ** 2 / 4 + om ** 2)
    lam[0] = 0.0
    shell = np.sort(lam)[:6]
    V0 = torch.tensor(np.random.default_rng(6).standard_normal((6, c.nd)), device=DEV)
    res = api.rpa_energy(dc, 6, [om], [1.0], [V0], dict(cocg_tol=1e-12, subspace_iters=60,
                                                         ec_tol=1e-14), save=True)
    C = res["Csave"][0][0].cpu().numpy()
    np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(C)), shell, rtol=1e-9)
    assert abs(res["E_c"][0] - np.sum(osub.g(shell)) / (2 * np.pi)) <= 1e-9 * abs(res["E_c"][0])


def test_backward_matches_oracle_adjoint():
    say("rpa_energy_backward 12^3 N_s=3 N_r=6 two frequencies")
    c = synth.small_cell(n=12, h=0.5, n_wells=2, n_occ=3, seed=11)
    dc = api.device_cell(c, DEV)
    # 0.1 lies below the default mixed_min_omega: that frequency's solves run the FP64 kernel
    # inside the mixed buffers, with complex solutions for the gradient epilogue
    om, W = np.array([2.0, 0.1]), np.array([0.6, 0.9])
    V0 = np.random.default_rng(6).standard_normal((6, c.nd))
    opts = dict(cocg_tol=1e-12, subspace_iters=3, ec_tol=0.0)
    res = api.rpa_energy(dc, 6, om, W, [torch.tensor(V0, device=DEV)], opts, save=True)
    grad, rc, st = api.rpa_energy_backward(dc, om, W, res["Vsave"][0], res["Csave"][0], 1.0, opts)
    assert rc == 0
    Vs = [res["Vsave"][0][m].cpu().numpy().T for m in range(2)]
    Cs = [res["Csave"][0][m].cpu().numpy() for m in range(2)]
    ref = ograd.energy_backward(c.vloc, c.psi.T, c.eps, c.shape, c.h, om, W, Vs, Cs, 1e-12, 5000)
    assert rel(grad.cpu().numpy(), ref) < 1e-8


# ---------------------------------------------------------------------------- mixed precision
MIXED = 1


def test_mixed_chi0_matches_oracle(wl0, dc0):
    c = wl0.cells[0]
    say("mixed chi0 12^3 16 vectors tol 1e-10")
    U = np.random.default_rng(2).standard_normal((16, c.nd))
    out, rc, st = api.rpa_apply_chi0(dc0, 1.0, torch.tensor(U, device=DEV),
                                     dict(cocg_tol=1e-10, precision=MIXED))
    ref, iters, _ = ochi0.chi0_apply(U.T, c.vloc, c.psi.T, c.eps, 1.0, c.shape, c.h, 1e-10, 5000)
    assert rc == 0 and st["n_unconverged"] == 0 and st["refinements"] >= 64
    assert rel(out.cpu().numpy().T, ref) < 1e-9


@pytest.mark.parametrize("omega", [0.02, 8.8])
def test_mixed_chi0_extreme_frequencies(wl0, dc0, omega):
    # Two solutions meeting a residual tolerance tol can differ by up to cond(A) * tol
    # (cond ~ 1e3 at omega = 0.02); the mixed path follows a different Krylov sequence from
    # the oracle, so both solve to 1e-12 and are compared at 1e-9.
    c = wl0.cells[0]
    say("mixed chi0 omega", omega)
    U = np.random.default_rng(3).standard_normal((4, c.nd))
    # mixed_min_omega = 0: complex64 at every frequency (the default solves omega = 0.02 in FP64)
    out, rc, st = api.rpa_apply_chi0(dc0, omega, torch.tensor(U, device=DEV),
                                     dict(cocg_tol=1e-12, precision=MIXED, mixed_min_omega=0.0))
    ref, _, _ = ochi0.chi0_apply(U.T, c.vloc, c.psi.T, c.eps, omega, c.shape, c.h, 1e-12, 5000)
    assert rc == 0 and rel(out.cpu().numpy().T, ref) < 1e-9 and st["refinements"] > 0


def test_mixed_path_solves_low_frequencies_in_fp64(wl0, dc0):
    # below options.mixed_min_omega (default 0.2) the mixed path runs the FP64 kernel on its
    # own buffers: the same recurrence as the FP64 path, so the same chi0 bit for bit, and no
    # complex64 refinements; above it, complex64 with refinements
    c = wl0.cells[0]
    thr = L.default_options().mixed_min_omega
    say("mixed path: FP64 below mixed_min_omega", thr)
    U = torch.tensor(np.random.default_rng(4).standard_normal((4, c.nd)), device=DEV)
    o = dict(cocg_tol=1e-10)
    for omega in (0.02, 0.98 * thr):
        mx, rc, st = api.rpa_apply_chi0(dc0, omega, U, dict(o, precision=MIXED))
        f64, rc2, st2 = api.rpa_apply_chi0(dc0, omega, U, o)
        assert rc == 0 and rc2 == 0 and st["refinements"] == 0
        assert torch.equal(mx, f64)
        assert st["cocg_iters_total"] == st2["cocg_iters_total"]
    mx, rc, st = api.rpa_apply_chi0(dc0, thr, U, dict(o, precision=MIXED))
    assert rc == 0 and st["refinements"] > 0
    # an explicit threshold moves the boundary
    mx, rc, st = api.rpa_apply_chi0(dc0, 0.05, U, dict(o, precision=MIXED, mixed_min_omega=0.05))
    assert rc == 0 and st["refinements"] > 0
    # a block whose vectors straddle the threshold (batched frequencies) splits into launches
    om, W = np.array([1.0, 0.03]), np.array([1.0, 1.0])
    V = torch.tensor(np.random.default_rng(5).standard_normal((4, c.nd)), device=DEV)
    ob = dict(o, subspace_iters=1, ec_tol=0.0, freq_mode=INDEPENDENT)
    e_mx = api.rpa_energy(dc0, 4, om, W, [V], dict(ob, precision=MIXED))
    e_64 = api.rpa_energy(dc0, 4, om, W, [V], ob)
    assert e_mx["stats"]["cocg_launches"] == 2 and e_mx["stats"]["refinements"] > 0
    assert e_mx["E_freq"][0][1] == e_64["E_freq"][0][1]
    assert abs(e_mx["E_freq"][0][0] - e_64["E_freq"][0][0]) <= 1e-9 * abs(e_64["E_freq"][0][0])


def test_mixed_energy_matches_oracle(wl0, dc0, oracle_e0):
    say("mixed rpa_energy 12^3")
    V0 = torch.tensor(wl0.V0[0], device=DEV)
    res = api.rpa_energy(dc0, 16, wl0.omegas, wl0.weights, [V0],
                         dict(cocg_tol=1e-10, subspace_iters=5, ec_tol=0.0, precision=MIXED))
    E = res["E_c"][0]
    say("E_c mixed %.15e oracle %.15e" % (E, oracle_e0["E_c"]))
    assert res["status"] == 0
    assert abs(E - oracle_e0["E_c"]) <= 1e-9 * abs(oracle_e0["E_c"])


def test_mixed_backward_matches_fp64():
    say("mixed backward vs fp64 backward 12^3")
    c = synth.small_cell(n=12, h=0.5, n_wells=2, n_occ=3, seed=11)
    dc = api.device_cell(c, DEV)
    # 0.1 lies below the default mixed_min_omega: that frequency's solves run the FP64 kernel
    # inside the mixed buffers, with complex solutions for the gradient epilogue
    om, W = np.array([2.0, 0.1]), np.array([0.6, 0.9])
    V0 = np.random.default_rng(6).standard_normal((6, c.nd))
    o64 = dict(cocg_tol=1e-11, subspace_iters=3, ec_tol=0.0)
    res = api.rpa_energy(dc, 6, om, W, [torch.tensor(V0, device=DEV)], o64, save=True)
    g64, _, _ = api.rpa_energy_backward(dc, om, W, res["Vsave"][0], res["Csave"][0], 1.0, o64)
    gmx, rc, st = api.rpa_energy_backward(dc, om, W, res["Vsave"][0], res["Csave"][0], 1.0,
                                          dict(o64, precision=MIXED))
    assert rc == 0 and st["refinements"] > 0
    assert rel(gmx.cpu().numpy(), g64.cpu().numpy()) < 1e-8


def test_mixed_capped_systems_continue_in_fp64(wl0, dc0):
    # At omega = 0.02 and tol 1e-10 the oracle needs at most 164 COCG steps, while the
    # complex64 recurrences of the two orbitals next to the gap need about 240-300; with the
    # cap at 180 those stop short and the library solves them on in FP64 from where they
    # stopped (x_hi, r_hi = b - A x_hi) to the same tolerance (a CPU emulation of both stages
    # puts the continuation at 60-135 steps).
    c = wl0.cells[0]
    say("mixed chi0 omega 0.02, cap 180: FP64 continuation of capped systems")
    U = np.random.default_rng(21).standard_normal((4, c.nd))
    ref, iters, _ = ochi0.chi0_apply(U.T, c.vloc, c.psi.T, c.eps, 0.02, c.shape, c.h, 1e-10,
                                     5000)
    assert iters.max() < 180
    out, rc, st = api.rpa_apply_chi0(dc0, 0.02, torch.tensor(U, device=DEV),
                                     dict(cocg_tol=1e-10, cocg_max_iter=180, precision=MIXED,
                                          mixed_min_omega=0.0))
    say("fallbacks", st["fp64_fallbacks"], "launches", st["cocg_launches"])
    assert rc == 0 and st["n_unconverged"] == 0 and st["fp64_fallbacks"] > 0
    assert st["cocg_launches"] == 2
    # the continuation restarts the Krylov space from x_hi, so its iterate is not the oracle's:
    # two solutions meeting tol 1e-10 differ by up to cond(A) tol ~ 1e-7 at this frequency
    assert rel(out.cpu().numpy().T, ref) < 1e-7
    # the backward's solves take the same route (complex solutions kept), same bound
    om, W = np.array([0.02]), np.array([1.0])
    V = np.linalg.qr(np.random.default_rng(22).standard_normal((c.nd, 4)))[0].T.copy()
    o = dict(cocg_tol=1e-10, subspace_iters=1, ec_tol=0.0)
    res = api.rpa_energy(dc0, 4, om, W, [torch.tensor(V, device=DEV)], o, save=True)
    g64, _, _ = api.rpa_energy_backward(dc0, om, W, res["Vsave"][0], res["Csave"][0], 1.0, o)
    gmx, rc2, st2 = api.rpa_energy_backward(dc0, om, W, res["Vsave"][0], res["Csave"][0], 1.0,
                                            dict(o, precision=MIXED, cocg_max_iter=180,
                                                 mixed_min_omega=0.0))
    say("backward fallbacks", st2["fp64_fallbacks"])
    assert rc2 == 0 and st2["n_unconverged"] == 0 and st2["fp64_fallbacks"] > 0
    assert rel(gmx.cpu().numpy(), g64.cpu().numpy()) < 1e-7


def test_mixed_breakdown_restarts_once_in_fp64(wl0, dc0, monkeypatch):
    # A breakdown threshold that no bilinear form passes makes every complex64 solve break down
    # at its first step: the kernel ends it with a reliable update (x_hi = 0, r_hi = b) and the
    # library restarts it once in FP64 from there, the same recurrence as the FP64 path.  A
    # threshold that trips part of the way restarts systems from a partial x_hi; compared with
    # the oracle at cond(A) tol, since the restart begins a new Krylov space.
    c = wl0.cells[0]
    ns = c.psi.shape[0]
    say("mixed chi0 with forced complex64 breakdowns: FP64 restart")
    U = np.random.default_rng(23).standard_normal((4, c.nd))
    Ut = torch.tensor(U, device=DEV)
    o = dict(cocg_tol=1e-10, precision=MIXED, mixed_min_omega=0.0)
    monkeypatch.setenv("RPA_MIXED_BD_TOL", "1e300")
    mx, rc, st = api.rpa_apply_chi0(dc0, 0.5, Ut, o)
    monkeypatch.delenv("RPA_MIXED_BD_TOL")
    f64, rc2, st2 = api.rpa_apply_chi0(dc0, 0.5, Ut, dict(cocg_tol=1e-10))
    say("first-step breakdowns: fallbacks", st["fp64_fallbacks"], "breakdowns", st["n_breakdown"])
    assert rc == 0 and rc2 == 0 and st["n_breakdown"] == 0 and st["fp64_fallbacks"] == 4 * ns
    assert rel(mx.cpu().numpy(), f64.cpu().numpy()) < 1e-12
    ref, _, _ = ochi0.chi0_apply(U.T, c.vloc, c.psi.T, c.eps, 0.5, c.shape, c.h, 1e-10, 5000)
    monkeypatch.setenv("RPA_MIXED_BD_TOL", "0.05")
    mx2, rc3, st3 = api.rpa_apply_chi0(dc0, 0.5, Ut, o)
    monkeypatch.delenv("RPA_MIXED_BD_TOL")
    say("breakdowns part of the way: fallbacks", st3["fp64_fallbacks"], "refinements",
        st3["refinements"])
    assert rc3 == 0 and st3["n_breakdown"] == 0 and st3["fp64_fallbacks"] > 0
    assert rel(mx2.cpu().numpy().T, ref) < 1e-7


# ---------------------------------------------------------------------------- batched frequencies
INDEPENDENT = 1


@pytest.fixture(scope="module")
def small3():
    c = synth.small_cell(n=12, h=0.5, n_wells=2, n_occ=3, seed=11)
    om, W = synth.frequency_rule(3)
    V0 = np.random.default_rng(8).standard_normal((6, c.nd))
    ref = oenergy.rpa_energy(c.vloc, c.psi.T, c.eps, c.shape, c.h, V0.T, om, W, 1e-11, 5000, 3,
                             mode="independent")
    return c, om, W, V0, ref


@pytest.mark.parametrize("precision", [0, MIXED])
def test_independent_frequencies_batched_match_oracle(small3, precision):
    # every frequency starts from V0; the GPU advances all three in one chi0 launch per
    # subspace iteration (per-system shifts), the oracle one frequency after the other
    c, om, W, V0, ref = small3
    say("batched independent frequencies, precision", precision)
    dc = api.device_cell(c, DEV)
    res = api.rpa_energy(dc, 6, om, W, [torch.tensor(V0, device=DEV)],
                         dict(cocg_tol=1e-11, subspace_iters=3, ec_tol=0.0,
                              freq_mode=INDEPENDENT, precision=precision), save=True)
    assert res["status"] == 0
    assert list(res["iters"][0]) == [3, 3, 3]
    np.testing.assert_allclose(res["E_freq"][0], ref["E_freq"], rtol=1e-9)
    assert abs(res["E_c"][0] - ref["E_c"]) <= 1e-9 * abs(ref["E_c"])
    # each saved (V_m, C_m) is the pair behind E_m
    for m in range(3):
        C = res["Csave"][0][m].cpu().numpy()
        mu = np.linalg.eigvalsh(0.5 * (C + C.T))
        # log-det route vs eigenvalue route: g(mu) ~ mu^2/2 loses ~eps/|mu| relative
        assert abs(W[m] * np.sum(osub.g(mu)) / (2 * np.pi) - res["E_freq"][0][m]) \
            <= 1e-10 * abs(res["E_freq"][0][m])
    # the backward consumes the batched saves like the warm ones
    grad, rc, _ = api.rpa_energy_backward(dc, om, W, res["Vsave"][0], res["Csave"][0], 1.0,
                                          dict(cocg_tol=1e-11))
    Vs = [res["Vsave"][0][m].cpu().numpy().T for m in range(3)]
    Cs = [res["Csave"][0][m].cpu().numpy() for m in range(3)]
    gref = ograd.energy_backward(c.vloc, c.psi.T, c.eps, c.shape, c.h, om, W, Vs, Cs, 1e-12, 5000)
    assert rc == 0 and rel(grad.cpu().numpy(), gref) < 1e-8


def test_independent_batched_stops_each_frequency_on_its_own(small3):
    # with an energy tolerance the frequencies stop at different counts; the result for each
    # equals a single-frequency run of the same length
    c, om, W, V0, _ = small3
    say("batched independent frequencies, per-frequency stopping")
    dc = api.device_cell(c, DEV)
    # (the oracle, same inputs: 40+, 16 and 14 iterations to a relative change of 1e-4, so
    # the highest frequency reaches the cap of 30 and is reported as capped)
    opts = dict(cocg_tol=1e-11, subspace_iters=30, ec_tol=1e-4, freq_mode=INDEPENDENT)
    res = api.rpa_energy(dc, 6, om, W, [torch.tensor(V0, device=DEV)], opts)
    its = res["iters"][0]
    capped = res["stats"]["subspace_capped"]
    say("subspace iterations", its, "capped", capped)
    assert its[0] == 30 and 2 <= its[1] < 30 and 2 <= its[2] < 30
    assert capped == 1 and res["status"] == L.RPA_ESUBCAP
    for m in range(3):
        one = api.rpa_energy(dc, 6, [om[m]], [W[m]], [torch.tensor(V0, device=DEV)],
                             dict(opts, subspace_iters=int(its[m]), ec_tol=0.0))
        assert abs(one["E_c"][0] - res["E_freq"][0][m]) <= 1e-9 * abs(one["E_c"][0])




@pytest.mark.parametrize("mode", [0, INDEPENDENT])
def test_subspace_cap_is_reported(small3, mode):
    # an energy tolerance no iterate can meet in 2 iterations: every frequency stops at the
    # cap, the energy of the last iterate is written, and the call says so (RPA_ESUBCAP with
    # the count in the stats); a fixed count (ec_tol = 0) is never a cap, and a loose
    # tolerance met before the cap is not one either
    c, om, W, V0, _ = small3
    say("subspace cap warning, mode", mode)
    dc = api.device_cell(c, DEV)
    V = torch.tensor(V0, device=DEV)
    base = dict(cocg_tol=1e-11, freq_mode=mode)
    capped = api.rpa_energy(dc, 6, om, W, [V], dict(base, subspace_iters=2, ec_tol=1e-15))
    assert capped["status"] == L.RPA_ESUBCAP
    assert capped["stats"]["subspace_capped"] == len(om)
    np.testing.assert_array_equal(capped["iters"][0], [2] * len(om))
    fixed = api.rpa_energy(dc, 6, om, W, [V], dict(base, subspace_iters=2, ec_tol=0.0))
    assert fixed["status"] == 0 and fixed["stats"]["subspace_capped"] == 0
    assert np.all(np.abs(fixed["E_freq"][0] - capped["E_freq"][0]) <= 1e-12 * np.abs(fixed["E_freq"][0]))
    loose = api.rpa_energy(dc, 6, om, W, [V], dict(base, subspace_iters=10, ec_tol=0.5))
    assert loose["status"] == 0 and loose["stats"]["subspace_capped"] == 0
    assert np.all(loose["iters"][0] >= 2) and np.all(loose["iters"][0] < 10)
    one = api.rpa_subspace_iter(dc, float(om[0]), float(W[0]), V.clone(),
                                dict(base, subspace_iters=3, ec_tol=1e-15), want_ritz=False,
                                want_saved=False)
    assert one["status"] == L.RPA_ESUBCAP and one["n_iter"] == 3
    assert one["stats"]["subspace_capped"] == 1


# ---------------------------------------------------------------------------- Gauss SQ energy
@pytest.mark.parametrize("n_o", [2, 4, 16])
def test_sq_energy_of_the_gpu_projected_matrix(wl0, dc0, n_o):
    # the GPU's SQ energy of its own C against the oracle's SQ on that same C; at order 16
    # (= N_r) the rule is exact and equals the Rayleigh-Ritz energy
    say("SQ energy, order", n_o)
    from oracle.subspace import chol_orthonormalize
    V = torch.tensor(chol_orthonormalize(wl0.V0[0].T).T.copy(), device=DEV)
    r = api.rpa_subspace_iter(dc0, 1.0, 0.7, V.clone(), dict(cocg_tol=1e-10, subspace_iters=1,
                                                            ec_tol=0.0, sq_order=n_o))
    C = r["C"].cpu().numpy()
    ref = osub.sq_energy(C, 0.7, n_o)
    assert abs(r["E"] - ref) <= 1e-12 * abs(ref)
    rr = 0.7 / (2 * np.pi) * np.sum(osub.g(np.linalg.eigvalsh(C)))
    if n_o == 16:
        assert abs(r["E"] - rr) <= 1e-12 * abs(rr)
    else:
        assert r["E"] >= rr - 1e-15      # Gauss SQ approaches from above (g'' < 0)


def test_energy_with_sq_matches_oracle(wl0, dc0):
    say("rpa_energy 12^3 with SQ order 3")
    c = wl0.cells[0]
    ref = oenergy.rpa_energy(c.vloc, c.psi.T, c.eps, c.shape, c.h, wl0.V0[0].T, wl0.omegas,
                             wl0.weights, 1e-10, 5000, 5, sq_order=3)
    res = api.rpa_energy(dc0, 16, wl0.omegas, wl0.weights, [torch.tensor(wl0.V0[0], device=DEV)],
                         dict(cocg_tol=1e-10, subspace_iters=5, ec_tol=0.0, sq_order=3))
    assert res["status"] == 0
    assert abs(res["E_c"][0] - ref["E_c"]) <= 1e-9 * abs(ref["E_c"])


def test_batched_frequencies_with_sq_match_oracle(small3):
    c, om, W, V0, _ = small3
    say("batched frequencies with SQ order 2")
    ref = oenergy.rpa_energy(c.vloc, c.psi.T, c.eps, c.shape, c.h, V0.T, om, W, 1e-11, 5000, 3,
                             mode="independent", sq_order=2)
    dc = api.device_cell(c, DEV)
    res = api.rpa_energy(dc, 6, om, W, [torch.tensor(V0, device=DEV)],
                         dict(cocg_tol=1e-11, subspace_iters=3, ec_tol=0.0, freq_mode=INDEPENDENT,
                              sq_order=2))
    np.testing.assert_allclose(res["E_freq"][0], ref["E_freq"], rtol=1e-9)


# ---------------------------------------------------------------------------- several cells
@pytest.mark.parametrize("mode,precision", [(0, 0), (1, MIXED)])
def test_several_cells_run_concurrently_and_match_single_calls(mode, precision):
    # uneven cells (one of them an isolated box) in one rpa_energy call run on their own
    # streams at the same time; each cell's result equals its own one-cell call bitwise
    say("three cells concurrently, mode", mode, "precision", precision)
    cells = [synth.small_cell(n=12, h=0.5, n_wells=2, n_occ=3, seed=11),
             synth.box_cell((12, 12, 13), 0.5, 2, 4, 21),
             synth.small_cell(n=14, h=0.45, n_wells=3, n_occ=5, seed=12)]
    nrs = [6, 8, 10]
    om, W = synth.frequency_rule(3)
    dcs = [api.device_cell(c, DEV) for c in cells]
    V0s = [torch.tensor(np.random.default_rng(20 + i).standard_normal((r, c.nd)), device=DEV)
           for i, (c, r) in enumerate(zip(cells, nrs))]
    opts = dict(cocg_tol=1e-10, subspace_iters=3, ec_tol=0.0, freq_mode=mode, precision=precision)
    res = api.rpa_energy(dcs, nrs, om, W, V0s, opts, save=True)
    assert res["status"] == 0
    for i in range(3):
        one = api.rpa_energy(dcs[i], nrs[i], om, W, [V0s[i]], opts, save=True)
        assert np.array_equal(one["E_freq"][0], res["E_freq"][i])
        assert torch.equal(one["Csave"][0], res["Csave"][i])
