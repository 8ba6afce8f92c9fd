"""Runs the oracle on all host cores: slices of a block (trial vectors, or the orbitals of one
trial vector) go to worker processes, each calling the oracle's own functions unchanged.
Test infrastructure only; nothing here computes beyond splitting work and summing the
per-orbital contributions chi0 u = 4 sum_n Re(psi_n x_n) that the oracle's chi0_apply sums
in the same way."""
import multiprocessing as mp
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np


def n_workers():
    return max(1, min(16, len(os.sched_getaffinity(0))))


def _one_thread():
    os.environ["OMP_NUM_THREADS"] = "1"
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:
        pass


def pool(n=None):
    """Worker processes started fresh (spawn): they import only numpy and the oracle."""
    return ProcessPoolExecutor(max_workers=n or n_workers(), mp_context=mp.get_context("spawn"),
                               initializer=_one_thread)


def _chi0_columns(args):
    from oracle import chi0
    U, vloc, psi, eps, om, shape, h, tol, max_iter = args
    out, it, st = chi0.chi0_apply(U, vloc, psi, eps, om, shape, h, tol, max_iter)
    return out, it, st


def chi0_apply(ex, U, vloc, psi, eps, om, shape, h, tol, max_iter):
    """oracle.chi0.chi0_apply(U, ...) with the columns of U spread over the pool."""
    nv = U.shape[1]
    k = min(nv, n_workers())
    cuts = np.linspace(0, nv, k + 1).astype(int)
    jobs = [(U[:, a:b], vloc, psi, eps, om, shape, h, tol, max_iter)
            for a, b in zip(cuts[:-1], cuts[1:]) if b > a]
    res = list(ex.map(_chi0_columns, jobs))
    # systems s = n + N_s j: contiguous column slices keep the global order
    return (np.concatenate([r[0] for r in res], axis=1), np.concatenate([r[1] for r in res]),
            np.concatenate([r[2] for r in res]))


def _orbital_systems(args):
    from oracle import chi0, cocg, fd
    u, vloc, psi, eps, om, shape, h, tol, max_iter, orbs = args
    bp, _ = chi0.build_rhs(u[:, None], psi, h ** 3)          # all N_s systems of this vector
    shifts = np.asarray(eps, dtype=np.float64)[orbs] + 1j * om
    x, it, st = cocg.cocg_batched(lambda v: fd.hamiltonian_apply(v, vloc, shape, h), shifts,
                                  -bp[:, orbs], tol, max_iter)
    out = np.zeros(u.shape[0])
    for t, n in enumerate(orbs):
        out += 4.0 * psi[:, n] * x[:, t].real
    return out, it, st


def chi0_column(ex, u, vloc, psi, eps, om, shape, h, tol, max_iter, orbitals=None):
    """chi0 applied to one trial vector u, its N_s Sternheimer systems spread over the pool
    (orbitals dealt round-robin, so the hardest ones, next to the gap, land on different
    workers); with `orbitals`, only those orbitals' terms 4 psi_n Re x_n (the column is the
    sum of the terms of all orbitals).  Returns (chi0 u or the partial sum, iterations per
    orbital, status per orbital; zero for orbitals not solved)."""
    ns = psi.shape[1]
    orbs = list(range(ns)) if orbitals is None else list(orbitals)
    k = min(len(orbs), n_workers())
    groups = [orbs[w::k] for w in range(k)]
    jobs = [(u, vloc, psi, eps, om, shape, h, tol, max_iter, g) for g in groups]
    out = np.zeros(u.shape[0])
    it = np.zeros(ns, dtype=np.int64)
    st = np.zeros(ns, dtype=np.int64)
    for g, (o, i, s) in zip(groups, ex.map(_orbital_systems, jobs)):
        out += o
        it[g] = i
        st[g] = s
    return out, it, st
