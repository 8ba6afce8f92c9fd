"""RPA correlation energy over all frequencies (oracle).

Eq. 10 with the frequency rule of Sec. 3 and the loop structure of Algorithm 1:
    E_c = sum_m E_{c,m},   frequencies from the highest to the lowest.
Two start-vector policies:
  warm        (the paper's, Sec. 3) the subspace found at one frequency starts the next;
  independent every frequency starts from the same orthonormalised V0, so frequencies
              are independent of one another (the form a batched launch can run at once).
The initial block V0 is orthonormalised once by the Cholesky step before use.
"""
import numpy as np

from . import chi0 as _chi0
from . import coulomb
from .subspace import chol_orthonormalize, subspace_iteration


def chi0_tilde_apply(V, vloc, psi, eps, omega, shape, h, tol, max_iter, bc="periodic"):
    """R = nu^{1/2} chi0(i omega) nu^{1/2} V (Algorithm 1, loop over trial vectors)."""
    U = coulomb.nu_apply(V, shape, h, power=1, bc=bc)
    D, iters, status = _chi0.chi0_apply(U, vloc, psi, eps, omega, shape, h, tol, max_iter, bc=bc)
    R = coulomb.nu_apply(D, shape, h, power=1, bc=bc)
    return R, dict(iters=iters, status=status)


def rpa_energy(vloc, psi, eps, shape, h, V0, omegas, weights, cocg_tol, cocg_max_iter,
               subspace_iters, ec_tol=0.0, mode="warm", sq_order=0, bc="periodic"):
    """Full E_c.  subspace_iters is the fixed count (ec_tol <= 0) or the cap (ec_tol > 0);
    it may be a scalar or one value per frequency.  Returns a dict with E_c, per-frequency
    energies, iteration counts, and the saved (V_m, C_m) per frequency."""
    nf = len(omegas)
    its = np.broadcast_to(np.asarray(subspace_iters), (nf,))
    Vstart = chol_orthonormalize(np.asarray(V0, dtype=np.float64))
    V = Vstart
    res = dict(E_freq=np.zeros(nf), n_iter=np.zeros(nf, dtype=int), V_saved=[], C_saved=[],
               mu=[], cocg_iters=[], history=[])
    for m in range(nf):
        if mode == "independent":
            V = Vstart
        om = float(omegas[m])

        def apply(Vb, om=om):
            return chi0_tilde_apply(Vb, vloc, psi, eps, om, shape, h, cocg_tol, cocg_max_iter, bc)

        out = subspace_iteration(apply, V, float(weights[m]), int(its[m]), ec_tol, sq_order)
        res["E_freq"][m] = out["E"]
        res["n_iter"][m] = out["n_iter"]
        res["V_saved"].append(out["V_saved"])
        res["C_saved"].append(out["C"])
        res["mu"].append(out["mu"])
        res["history"].append(out["history"])
        res["cocg_iters"].append([i["iters"] for i in out["infos"]])
        V = out["V_next"]
    res["E_c"] = float(np.sum(res["E_freq"]))
    return res
