"""Tensor-level binding of the C ABI: the same five entry points, taking torch tensors.

This layer only marshals arguments: it allocates outputs and the workspace with torch
(device memory), passes raw pointers and the current HIP stream, and raises on negative
status codes.  Every step of the computation runs in the gfx950 kernels of
librpa_gfx950.so; there is no CPU fallback.

Tensor conventions: a block of k grid vectors is a (k, N_d) float64 tensor whose row j is
the grid vector j (that is the ABI's column-major N_d x k block); small matrices are
(m, m) float64 tensors holding the column-major matrix (symmetric ones are unaffected).
"""
import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import lib as _L


@dataclass
class DeviceCell:
    """A cell whose arrays live on the GPU (eps stays on the host, as the ABI requires)."""
    shape: tuple
    h: float
    vloc: torch.Tensor      # (N_d,) float64 device
    psi: torch.Tensor       # (N_s, N_d) float64 device
    eps: np.ndarray         # (N_s,) float64 host
    bc: int = 0             # RPA_BC_PERIODIC or RPA_BC_DIRICHLET

    @property
    def nd(self):
        return int(np.prod(self.shape))

    @property
    def n_occ(self):
        return int(self.psi.shape[0])

    def c_struct(self):
        c = _L.RpaCell()
        c.n[0], c.n[1], c.n[2] = (int(v) for v in self.shape)
        c.n_occ = self.n_occ
        c.h = float(self.h)
        c.v_loc = self.vloc.data_ptr()
        c.psi = self.psi.data_ptr()
        self._eps_c = np.ascontiguousarray(self.eps, dtype=np.float64)
        c.eps = self._eps_c.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        c.bc = int(self.bc)
        return c


def device_cell(cell, device="cuda"):
    """Upload a synth.Cell (or any object with shape, h, vloc, psi, eps) to the device."""
    return DeviceCell(tuple(cell.shape), float(cell.h),
                      torch.as_tensor(np.ascontiguousarray(cell.vloc), dtype=torch.float64,
                                      device=device),
                      torch.as_tensor(np.ascontiguousarray(cell.psi), dtype=torch.float64,
                                      device=device),
                      np.ascontiguousarray(cell.eps, dtype=np.float64),
                      _L.RPA_BC_DIRICHLET if getattr(cell, "bc", "periodic") == "dirichlet"
                      else _L.RPA_BC_PERIODIC)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _opts(opts):
    if opts is None:
        return _L.default_options()
    if isinstance(opts, dict):
        return _L.default_options(**opts)
    return opts


def workspace_size(op, cells, nvec, nfreq=1, opts=None):
    cells = cells if isinstance(cells, (list, tuple)) else [cells]
    nvec = nvec if isinstance(nvec, (list, tuple)) else [nvec]
    arr = (_L.RpaCell * len(cells))(*[c.c_struct() for c in cells])
    nv = (ctypes.c_int32 * len(nvec))(*nvec)
    out = ctypes.c_size_t(0)
    o = _opts(opts)
    _L.check(_L.load().rpa_workspace_size(op, len(cells), arr, nv, nfreq, ctypes.byref(o),
                                          ctypes.byref(out)), "rpa_workspace_size")
    return int(out.value)


def _workspace(nbytes, device):
    n = max(256, int(nbytes) + 256)
    buf = torch.empty(n, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf, buf.data_ptr() + off, n - off


def _check_block(X, nd, name):
    if X.dtype != torch.float64 or not X.is_cuda or not X.is_contiguous() or X.dim() != 2 \
            or X.shape[1] != nd:
        raise ValueError("%s must be a contiguous CUDA float64 tensor of shape (k, %d)" % (name, nd))


def rpa_apply_coulomb(cell, X, power=1, out=None):
    """nu^{power/2} X (Kronecker scheme); X is (k, N_d)."""
    _check_block(X, cell.nd, "X")
    k = X.shape[0]
    out = torch.empty_like(X) if out is None else out
    c = cell.c_struct()
    need = workspace_size(_L.RPA_OP_COULOMB, cell, k)
    keep, ws, nbytes = _workspace(need, X.device)
    _L.check(_L.load().rpa_apply_coulomb(ctypes.byref(c), power, k, X.data_ptr(), out.data_ptr(),
                                         ws, nbytes, _stream()), "rpa_apply_coulomb")
    del keep
    return out


def rpa_apply_coulomb_noalloc(cell, X, power=1, out=None):
    """nu^{power/2} X through the allocation-free entry point (the library's static device
    scratch, no workspace); out must be preallocated by the caller when given."""
    _check_block(X, cell.nd, "X")
    k = X.shape[0]
    out = torch.empty_like(X) if out is None else out
    c = cell.c_struct()
    _L.check(_L.load().rpa_apply_coulomb_noalloc(ctypes.byref(c), power, k, X.data_ptr(),
                                                 out.data_ptr(), _stream()),
             "rpa_apply_coulomb_noalloc")
    return out


def rpa_apply_chi0(cell, omega, X, opts=None):
    """chi0(i omega) X by DFPT/COCG; returns (out, status, stats dict)."""
    _check_block(X, cell.nd, "X")
    k = X.shape[0]
    out = torch.empty_like(X)
    c = cell.c_struct()
    o = _opts(opts)
    st = _L.RpaStats()
    need = workspace_size(_L.RPA_OP_CHI0, cell, k, opts=o)
    keep, ws, nbytes = _workspace(need, X.device)
    rc = _L.check(_L.load().rpa_apply_chi0(ctypes.byref(c), float(omega), k, X.data_ptr(),
                                           out.data_ptr(), ctypes.byref(o), ctypes.byref(st), ws,
                                           nbytes, _stream()), "rpa_apply_chi0")
    del keep
    return out, rc, st.as_dict()


def rpa_subspace_iter(cell, omega, weight, V, opts=None, want_ritz=True, want_saved=True):
    """Algorithm 1's subspace iteration at one frequency.  V (N_r, N_d) is updated in place.
    Returns dict(E, n_iter, ritz, V_saved, C, status, stats)."""
    _check_block(V, cell.nd, "V")
    nr = V.shape[0]
    c = cell.c_struct()
    o = _opts(opts)
    st = _L.RpaStats()
    Vs = torch.empty_like(V) if want_saved else None
    C = torch.empty((nr, nr), dtype=torch.float64, device=V.device) if want_saved else None
    ritz = np.zeros(nr) if want_ritz else None
    E = ctypes.c_double(0.0)
    nit = ctypes.c_int32(0)
    need = workspace_size(_L.RPA_OP_SUBSPACE, cell, nr, opts=o)
    keep, ws, nbytes = _workspace(need, V.device)
    rc = _L.check(_L.load().rpa_subspace_iter(
        ctypes.byref(c), float(omega), float(weight), nr, V.data_ptr(),
        Vs.data_ptr() if Vs is not None else None, C.data_ptr() if C is not None else None,
        ritz.ctypes.data_as(_L.PD) if ritz is not None else None, ctypes.byref(E),
        ctypes.byref(nit), ctypes.byref(o), ctypes.byref(st), ws, nbytes, _stream()),
        "rpa_subspace_iter")
    del keep
    return dict(E=E.value, n_iter=nit.value, ritz=ritz, V_saved=Vs, C=C, status=rc,
                stats=st.as_dict())


def rpa_energy(cells, nr, omegas, weights, V0, opts=None, save=False):
    """E_c for one or several cells.  V0: list of (N_r, N_d) device tensors.
    Returns dict(E_c (per cell), E_freq (ncell, nfreq), iters, Vsave, Csave, status, stats)."""
    cells = cells if isinstance(cells, (list, tuple)) else [cells]
    nr = list(nr) if isinstance(nr, (list, tuple)) else [nr]
    V0 = list(V0) if isinstance(V0, (list, tuple)) else [V0]
    nc, nf = len(cells), len(omegas)
    for c, V, r in zip(cells, V0, nr):
        _check_block(V, c.nd, "V0")
        if V.shape[0] != r:
            raise ValueError("V0 width does not match nr")
    structs = (_L.RpaCell * nc)(*[c.c_struct() for c in cells])
    o = _opts(opts)
    st = _L.RpaStats()
    om = np.ascontiguousarray(omegas, dtype=np.float64)
    wt = np.ascontiguousarray(weights, dtype=np.float64)
    nr_c = (ctypes.c_int32 * nc)(*nr)
    v0p = (ctypes.c_void_p * nc)(*[V.data_ptr() for V in V0])
    Vsave = Csave = None
    vsp = csp = None
    if save:
        Vsave = [torch.empty((nf, r, c.nd), dtype=torch.float64, device=V0[0].device)
                 for c, r in zip(cells, nr)]
        Csave = [torch.empty((nf, r, r), dtype=torch.float64, device=V0[0].device) for r in nr]
        vsp = (ctypes.c_void_p * nc)(*[t.data_ptr() for t in Vsave])
        csp = (ctypes.c_void_p * nc)(*[t.data_ptr() for t in Csave])
    ec = np.zeros(nc)
    ecf = np.zeros((nc, nf))
    its = np.zeros((nc, nf), dtype=np.int32)
    need = workspace_size(_L.RPA_OP_ENERGY, cells, nr, nf, o)
    keep, ws, nbytes = _workspace(need, V0[0].device)
    rc = _L.check(_L.load().rpa_energy(
        nc, structs, nr_c, nf, om.ctypes.data_as(_L.PD), wt.ctypes.data_as(_L.PD), v0p, vsp, csp,
        ctypes.byref(o), ec.ctypes.data_as(_L.PD), ecf.ctypes.data_as(_L.PD),
        its.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(st), ws, nbytes,
        _stream()), "rpa_energy")
    del keep
    return dict(E_c=ec, E_freq=ecf, iters=its, Vsave=Vsave, Csave=Csave, status=rc,
                stats=st.as_dict())


def rpa_energy_backward(cell, omegas, weights, Vsave, Csave, grad_ec=1.0, opts=None):
    """grad_ec * dE_c/dV_loc (N_d,) with orbitals, eigenvalues and saved subspaces fixed."""
    nf = len(omegas)
    nr = Vsave.shape[1]
    if Vsave.shape != (nf, nr, cell.nd) or Csave.shape != (nf, nr, nr):
        raise ValueError("Vsave/Csave shapes do not match")
    c = cell.c_struct()
    o = _opts(opts)
    st = _L.RpaStats()
    om = np.ascontiguousarray(omegas, dtype=np.float64)
    wt = np.ascontiguousarray(weights, dtype=np.float64)
    grad = torch.empty(cell.nd, dtype=torch.float64, device=Vsave.device)
    need = workspace_size(_L.RPA_OP_BACKWARD, cell, nr, nf, o)
    keep, ws, nbytes = _workspace(need, Vsave.device)
    rc = _L.check(_L.load().rpa_energy_backward(
        ctypes.byref(c), nf, om.ctypes.data_as(_L.PD), wt.ctypes.data_as(_L.PD), nr,
        Vsave.data_ptr(), Csave.data_ptr(), float(grad_ec), grad.data_ptr(), ctypes.byref(o),
        ctypes.byref(st), ws, nbytes, _stream()), "rpa_energy_backward")
    del keep
    return grad, rc, st.as_dict()


class RPAEnergy(torch.autograd.Function):
    """E_c as a differentiable function of V_loc (orbitals, eigenvalues and the subspaces
    found by the forward held fixed): forward = rpa_energy (saving V_m, C_m), backward =
    rpa_energy_backward with the incoming gradient as grad_ec.

        E = RPAEnergy.apply(vloc, cell, nr, omegas, weights, V0, opts)

    vloc: (N_d,) float64 device tensor (requires_grad as needed); cell: a DeviceCell whose
    psi, eps, shape and h are used (its vloc is replaced by the argument); V0: (nr, N_d).
    Returns a 0-d float64 tensor on the device of vloc."""

    @staticmethod
    def forward(ctx, vloc, cell, nr, omegas, weights, V0, opts=None):
        dc = DeviceCell(cell.shape, cell.h, vloc.detach().contiguous(), cell.psi, cell.eps,
                        cell.bc)
        res = rpa_energy(dc, nr, omegas, weights, V0, opts, save=True)
        ctx.dc, ctx.omegas, ctx.weights, ctx.opts = dc, list(omegas), list(weights), opts
        ctx.save_for_backward(res["Vsave"][0], res["Csave"][0])
        return torch.tensor(float(res["E_c"][0]), dtype=torch.float64, device=vloc.device)

    @staticmethod
    def backward(ctx, grad_out):
        Vs, Cs = ctx.saved_tensors
        g, _, _ = rpa_energy_backward(ctx.dc, ctx.omegas, ctx.weights, Vs, Cs,
                                      float(grad_out), ctx.opts)
        return g, None, None, None, None, None, None
