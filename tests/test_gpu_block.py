"""GPU parity of block COCG (options.cocg_block: the systems of one orbital and one frequency
solved as blocks with a shared Krylov space, with or without the Kronecker preconditioner)
against the oracle's block COCG and its plain DFPT, element by element: widths 2, 3, 4 and 8,
ragged blocks, chunked launches, an isolated box, a zero column and the iteration cap, equal
trial vectors (split blocks), the batched-frequency energy with its backward, row-slab steps
with the GEMM preconditioner passes, the gathered step where no march shape fits, and the
24^3 cell against the plain solver and the oracle's plain DFPT."""
import numpy as np
import pytest
import torch

import oracle_pool
from oracle import chi0 as ochi0
from oracle import energy as oenergy
from oracle import gradient as ograd
from oracle import fd as ofd
from oracle.block import bcocg, blocks_of, chi0_apply_block
from oracle.chi0 import build_rhs
from oracle.precond import kron_laplacian_inverse, precond_shift
from paper_2504_01816_amd import api, synth
from paper_2504_01816_amd import lib as L

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
PRE = L.RPA_FLAG_PRECOND


def say(*a):
    print(*a, flush=True)


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def oracle_splits(U, c, width, pre, omega, bc="periodic"):
    """Whether any block of the oracle's solve splits: its iteration counts change when the
    oracle solves the same blocks again with splitting disabled (pivot threshold 0)."""
    psi = c.psi.T
    ns = psi.shape[1]
    bp, _ = build_rhs(U.T, psi, c.h ** 3)
    for blk in blocks_of(np.full(U.shape[0], omega), width):
        for n in range(ns):
            cols = [n + ns * j for j in blk]
            shift = c.eps[n] + 1j * omega

            def A(P, shift=shift):
                return ofd.hamiltonian_apply(P, c.vloc, c.shape, c.h, bc=bc) - shift * P

            M = None
            if pre:
                ks = precond_shift(c.vloc, c.eps[n]) - 1j * omega

                def M(R, ks=ks):
                    return kron_laplacian_inverse(R, c.shape, c.h, np.full(R.shape[1], ks), bc=bc)

            _, it_a, _ = bcocg(A, -bp[:, cols], 1e-12, 5000, M)
            _, it_b, _ = bcocg(A, -bp[:, cols], 1e-12, 5000, M, split_tol=0.0)
            if np.any(it_a != it_b):
                return True
    return False


def iters_close(st, it_ref, split):
    # the same recurrence: without a split the totals agree to one step per system; a block
    # splits when a scaled pivot falls below the threshold, and near the threshold the
    # reduction order moves the split by a step or more (the oracle's own totals move with its
    # BLAS thread count there), so with a split the totals agree to 5%
    d = abs(st["cocg_iters_total"] - int(it_ref.sum()))
    return d <= (max(it_ref.size, 0.05 * it_ref.sum()) if split else it_ref.size)


@pytest.fixture(scope="module")
def wl0():
    return synth.workload(0)


@pytest.fixture(scope="module")
def dc0(wl0):
    return api.device_cell(wl0.cells[0], DEV)


@pytest.mark.parametrize("width,pre,omega", [(4, True, 1.0), (2, False, 0.02), (8, True, 0.02),
                                             (3, False, 8.8)])
def test_block_chi0_matches_oracle(wl0, dc0, width, pre, omega):
    c = wl0.cells[0]
    say("block chi0 12^3 width", width, "precond", pre, "omega", omega)
    U = np.random.default_rng(41).standard_normal((6, c.nd))
    o = dict(cocg_tol=1e-12, cocg_block=width, flags=PRE if pre else 0)
    out, rc, st = api.rpa_apply_chi0(dc0, omega, torch.tensor(U, device=DEV), o)
    ref, it_ref, st_ref = chi0_apply_block(U.T, c.vloc, c.psi.T, c.eps, omega, c.shape, c.h,
                                           1e-12, 5000, width, precond=pre)
    plain, it_plain, _ = ochi0.chi0_apply(U.T, c.vloc, c.psi.T, c.eps, omega, c.shape, c.h,
                                          1e-12, 5000)
    say("iterations gpu %d oracle %d single-system cocg %d" % (
        st["cocg_iters_total"], it_ref.sum(), it_plain.sum()))
    assert rc == 0 and st["n_unconverged"] == 0 and np.all(st_ref == 0)
    assert rel(out.cpu().numpy().T, ref) < 1e-9
    assert rel(out.cpu().numpy().T, plain) < 1e-9
    split = oracle_splits(U, c, width, pre, omega)
    say("a block splits: %s" % split)
    assert iters_close(st, it_ref, split)
    # single systems near the real axis drift by a few steps with the rounding order
    assert abs(st["cocg_iters_max"] - int(it_ref.max())) <= max(2, 0.05 * it_ref.max())


def test_block_chunked_launches_match_oracle_per_chunk(wl0, dc0):
    c = wl0.cells[0]
    ns = c.psi.shape[0]
    say("block chi0 in two launches of 4 vectors, width 3")
    U = np.random.default_rng(42).standard_normal((8, c.nd))
    o = dict(cocg_tol=1e-12, cocg_block=3, max_systems=4 * ns, flags=PRE)
    out, rc, st = api.rpa_apply_chi0(dc0, 0.5, torch.tensor(U, device=DEV), o)
    assert rc == 0 and st["cocg_launches"] == 2
    for j0 in (0, 4):
        ref, _, _ = chi0_apply_block(U[j0:j0 + 4].T, c.vloc, c.psi.T, c.eps, 0.5, c.shape, c.h,
                                     1e-12, 5000, 3, precond=True)
        assert rel(out[j0:j0 + 4].cpu().numpy().T, ref) < 1e-9


def test_block_box_matches_oracle():
    c = synth.box_cell((12, 12, 13), 0.5, 2, 4, 21)
    dc = api.device_cell(c, DEV)
    say("block chi0 isolated box, width 4")
    U = np.random.default_rng(43).standard_normal((5, c.nd))
    for omega, pre in ((1.0, True), (0.05, False)):
        out, rc, st = api.rpa_apply_chi0(dc, omega, torch.tensor(U, device=DEV),
                                         dict(cocg_tol=1e-12, cocg_block=4,
                                              flags=PRE if pre else 0))
        ref, it_ref, _ = chi0_apply_block(U.T, c.vloc, c.psi.T, c.eps, omega, c.shape, c.h,
                                          1e-12, 5000, 4, precond=pre, bc="dirichlet")
        assert rc == 0 and rel(out.cpu().numpy().T, ref) < 1e-9
        assert iters_close(st, it_ref, oracle_splits(U, c, 4, pre, omega, bc="dirichlet"))


def test_block_zero_column_and_iteration_cap(wl0, dc0):
    c = wl0.cells[0]
    say("block chi0 cap 3, zero column, width 4")
    U = np.random.default_rng(44).standard_normal((4, c.nd))
    U[1] = 0.0
    out, rc, st = api.rpa_apply_chi0(dc0, 0.5, torch.tensor(U, device=DEV),
                                     dict(cocg_max_iter=3, cocg_block=4, flags=PRE))
    ref, it_ref, st_ref = chi0_apply_block(U.T, c.vloc, c.psi.T, c.eps, 0.5, c.shape, c.h,
                                           1e-8, 3, 4, precond=True)
    assert rc == 1 and st["n_unconverged"] == int((st_ref == 1).sum())
    assert st["n_unconverged"] == 3 * c.psi.shape[0]
    assert st["cocg_iters_max"] == 3
    assert float(out[1].abs().max()) == 0.0
    assert rel(out.cpu().numpy().T, ref) < 1e-11


def test_block_with_equal_vectors_splits_and_matches_oracle(wl0, dc0):
    # two equal trial vectors give every orbital's block two equal right-hand sides: the block
    # is rank deficient from the first step and splits into single-vector solves
    c = wl0.cells[0]
    say("block chi0 with equal vectors (split), width 4")
    U = np.random.default_rng(47).standard_normal((4, c.nd))
    U[3] = U[1]
    for pre in (True, False):
        o = dict(cocg_tol=1e-12, cocg_block=4, flags=PRE if pre else 0)
        out, rc, st = api.rpa_apply_chi0(dc0, 0.3, torch.tensor(U, device=DEV), o)
        ref, it_ref, _ = chi0_apply_block(U.T, c.vloc, c.psi.T, c.eps, 0.3, c.shape, c.h,
                                          1e-12, 5000, 4, precond=pre)
        plain, _, _ = ochi0.chi0_apply(U.T, c.vloc, c.psi.T, c.eps, 0.3, c.shape, c.h, 1e-12,
                                       5000)
        o_np = out.cpu().numpy()
        assert rc == 0 and rel(o_np.T, ref) < 1e-9 and rel(o_np.T, plain) < 1e-9
        assert rel(o_np[3], o_np[1]) < 1e-12
        assert iters_close(st, it_ref, True)             # equal columns: every block splits


def test_block_batched_energy_and_backward_match_oracle():
    c = synth.small_cell(n=12, h=0.5, n_wells=2, n_occ=3, seed=11)
    dc = api.device_cell(c, DEV)
    say("block energy (batched frequencies, width 4) + backward")
    om, W = np.array([2.0, 0.3]), np.array([0.6, 0.9])
    V0 = np.random.default_rng(45).standard_normal((6, c.nd))
    o = dict(cocg_tol=1e-12, subspace_iters=2, ec_tol=0.0, freq_mode=L.RPA_INDEPENDENT,
             cocg_block=4, flags=PRE)
    ref = oenergy.rpa_energy(c.vloc, c.psi.T, c.eps, c.shape, c.h, V0.T, om, W, 1e-12, 5000, 2,
                             mode="independent")
    res = api.rpa_energy(dc, 6, om, W, [torch.tensor(V0, device=DEV)], o, save=True)
    assert res["status"] == 0
    np.testing.assert_allclose(res["E_freq"][0], ref["E_freq"], rtol=1e-9)
    grad, rc, st = api.rpa_energy_backward(dc, om, W, res["Vsave"][0], res["Csave"][0], 1.0, o)
    Vs = [res["Vsave"][0][m].cpu().numpy().T for m in range(2)]
    Cs = [res["Csave"][0][m].cpu().numpy() for m in range(2)]
    gref = ograd.energy_backward(c.vloc, c.psi.T, c.eps, c.shape, c.h, om, W, Vs, Cs, 1e-12, 5000)
    assert rc == 0 and rel(grad.cpu().numpy(), gref) < 1e-8


@pytest.fixture(scope="module")
def cell24_block():
    # the benchmark's 24^3 cell, a block of 64 trial vectors, and the oracle's plain DFPT chi0
    # (Eqs. 7-9, its own COCG) of two of them, computed once on the host cores
    wl = synth.workload(1, device=DEV)
    c = wl.cells[0]
    dc = api.device_cell(c, DEV)
    Un = np.random.default_rng(46).standard_normal((64, c.nd))
    pick = [5, 46]
    say("oracle chi0 24^3, vectors", pick)
    with oracle_pool.pool() as ex:
        ref, _, _ = oracle_pool.chi0_apply(ex, Un[pick].T, c.vloc, c.psi.T, c.eps, 0.69, c.shape,
                                           c.h, 1e-10, 5000)
    return dict(c=c, dc=dc, U=torch.tensor(Un, device=DEV), pick=pick, ref=ref)


@pytest.mark.parametrize("width,pre", [(4, True), (4, False)])
def test_block_cell24_matches_single_system_solver(cell24_block, width, pre):
    # the benchmark's 24^3 cell and block of 64 trial vectors (1024 systems, 256 blocks of 4):
    # block and single-system solves of the same systems give the same chi0 to the solver
    # tolerance; every block is checked, through the output columns of every vector, and two
    # columns of both against the oracle's plain DFPT (two solutions meeting tol 1e-10 differ
    # by up to cond(A) tol, about 1e-8 at this frequency)
    dc, U = cell24_block["dc"], cell24_block["U"]
    say("block chi0 24^3, 64 vectors, width", width, "precond", pre)
    base = dict(cocg_tol=1e-10)
    a, rc_a, st_a = api.rpa_apply_chi0(dc, 0.69, U, base)
    b, rc_b, st_b = api.rpa_apply_chi0(dc, 0.69, U, dict(base, cocg_block=width,
                                                         flags=PRE if pre else 0))
    say("iterations single %d block %d" % (st_a["cocg_iters_total"], st_b["cocg_iters_total"]))
    assert rc_a == 0 and rc_b == 0
    assert rel(b.cpu().numpy(), a.cpu().numpy()) < 1e-7
    pick, ref = cell24_block["pick"], cell24_block["ref"]
    for out in (a, b):
        assert rel(out[pick].cpu().numpy().T, ref) < 1e-7


def test_block_on_row_slabs_and_gemm_preconditioner():
    # a 36x36x12 cell: the plane exceeds one workgroup, so q = A p runs on row slabs, and the
    # axes beyond 32 points take the Kronecker GEMM passes of the preconditioner; two chunks
    c = synth._cell_from_seed((36, 36, 12), 0.45, 3, 3, 37, device=DEV)
    dc = api.device_cell(c, DEV)
    ns = c.psi.shape[0]
    say("block chi0 36x36x12 (row slabs, GEMM preconditioner passes), width 3, two chunks")
    U = np.random.default_rng(48).standard_normal((5, c.nd))
    out, rc, st = api.rpa_apply_chi0(dc, 0.3, torch.tensor(U, device=DEV),
                                     dict(cocg_tol=1e-12, cocg_block=3, flags=PRE,
                                          max_systems=3 * ns))
    assert rc == 0 and st["cocg_launches"] == 2
    for j0, j1 in ((0, 3), (3, 5)):
        ref, it_ref, _ = chi0_apply_block(U[j0:j1].T, c.vloc, c.psi.T, c.eps, 0.3, c.shape, c.h,
                                          1e-12, 5000, 3, precond=True)
        assert rel(out[j0:j1].cpu().numpy().T, ref) < 1e-9


def test_gathered_step_on_a_plane_no_march_shape_fits():
    # a 37x37 plane fits neither one workgroup (1369 columns) nor equal row slabs (37 is
    # prime), so q = A p takes the gathered step kernel; single-system and block solves
    c = synth._cell_from_seed((37, 37, 12), 0.45, 3, 3, 53, device=DEV)
    dc = api.device_cell(c, DEV)
    say("preconditioned and block chi0 on 37x37x12 (gathered step)")
    U = np.random.default_rng(49).standard_normal((3, c.nd))
    from oracle import precond as opre
    out, rc, st = api.rpa_apply_chi0(dc, 0.4, torch.tensor(U, device=DEV),
                                     dict(cocg_tol=1e-12, flags=PRE))
    ref, it_ref, _ = opre.chi0_apply_precond(U.T, c.vloc, c.psi.T, c.eps, 0.4, c.shape, c.h,
                                             1e-12, 5000)
    assert rc == 0 and rel(out.cpu().numpy().T, ref) < 1e-9
    assert abs(st["cocg_iters_total"] - int(it_ref.sum())) <= it_ref.size
    out, rc, st = api.rpa_apply_chi0(dc, 0.4, torch.tensor(U, device=DEV),
                                     dict(cocg_tol=1e-12, flags=PRE, cocg_block=3))
    ref, it_ref, _ = chi0_apply_block(U.T, c.vloc, c.psi.T, c.eps, 0.4, c.shape, c.h, 1e-12,
                                      5000, 3, precond=True)
    assert rc == 0 and rel(out.cpu().numpy().T, ref) < 1e-9
    assert iters_close(st, it_ref, oracle_splits(U, c, 3, True, 0.4))
