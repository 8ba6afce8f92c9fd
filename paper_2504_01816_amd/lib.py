"""ctypes view of the C ABI in include/rpa.h (librpa_gfx950.so, built in-tree).

No fallback exists: if the shared library is missing, load() raises.  Nothing here
computes anything; see api.py for the tensor-level wrappers.
"""
import ctypes
import os
from ctypes import POINTER, c_double, c_int32, c_int64, c_size_t, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("RPA_LIB_PATH") or os.path.join(HERE, "librpa_gfx950.so")

RPA_OK, RPA_ENOTCONV, RPA_ESUBCAP = 0, 1, 2
RPA_EINVAL, RPA_EWORKSPACE, RPA_EBREAKDOWN, RPA_ENOTPD, RPA_EHIP, RPA_ENOTIMPL = -1, -2, -3, -4, -5, -6
RPA_FP64, RPA_MIXED = 0, 1
RPA_WARM, RPA_INDEPENDENT = 0, 1
RPA_FLAG_PRECOND = 1
RPA_BC_PERIODIC, RPA_BC_DIRICHLET = 0, 1
RPA_OP_COULOMB, RPA_OP_CHI0, RPA_OP_SUBSPACE, RPA_OP_ENERGY, RPA_OP_BACKWARD = 0, 1, 2, 3, 4


class RpaCell(ctypes.Structure):
    _fields_ = [("n", c_int32 * 3), ("n_occ", c_int32), ("h", c_double),
                ("v_loc", c_void_p), ("psi", c_void_p), ("eps", POINTER(c_double)),
                ("bc", c_int32)]


class RpaOptions(ctypes.Structure):
    _fields_ = [("precision", c_int32), ("cocg_max_iter", c_int32), ("cocg_tol", c_double),
                ("subspace_iters", c_int32), ("freq_mode", c_int32), ("ec_tol", c_double),
                ("refine_tol", c_double), ("max_systems", c_int32), ("flags", c_int32),
                ("sq_order", c_int32), ("cocg_block", c_int32), ("mixed_min_omega", c_double)]


class RpaStats(ctypes.Structure):
    _fields_ = [("cocg_iters_total", c_int64), ("cocg_systems", c_int64),
                ("cocg_iters_max", c_int32), ("n_unconverged", c_int32),
                ("n_breakdown", c_int32), ("refinements", c_int32),
                ("chi0_applies", c_int32), ("subspace_iters_total", c_int32),
                ("cocg_launches", c_int64), ("cocg_kernel_ms", c_double),
                ("cocg_point_iters", c_double), ("fp64_fallbacks", c_int32),
                ("subspace_capped", c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


PD = POINTER(c_double)
PPD = POINTER(c_void_p)

_SIGS = {
    "rpa_version": (c_int32, []),
    "rpa_error_string": (ctypes.c_char_p, [c_int32]),
    "rpa_last_error": (ctypes.c_char_p, []),
    "rpa_default_options": (c_int32, [POINTER(RpaOptions)]),
    "rpa_workspace_size": (c_int32, [c_int32, c_int32, POINTER(RpaCell), POINTER(c_int32),
                                     c_int32, POINTER(RpaOptions), POINTER(c_size_t)]),
    "rpa_apply_coulomb": (c_int32, [POINTER(RpaCell), c_int32, c_int32, c_void_p, c_void_p,
                                    c_void_p, c_size_t, c_void_p]),
    "rpa_apply_coulomb_noalloc": (c_int32, [POINTER(RpaCell), c_int32, c_int32, c_void_p,
                                            c_void_p, c_void_p]),
    "rpa_apply_chi0": (c_int32, [POINTER(RpaCell), c_double, c_int32, c_void_p, c_void_p,
                                 POINTER(RpaOptions), POINTER(RpaStats), c_void_p, c_size_t,
                                 c_void_p]),
    "rpa_subspace_iter": (c_int32, [POINTER(RpaCell), c_double, c_double, c_int32, c_void_p,
                                    c_void_p, c_void_p, PD, PD, POINTER(c_int32),
                                    POINTER(RpaOptions), POINTER(RpaStats), c_void_p, c_size_t,
                                    c_void_p]),
    "rpa_energy": (c_int32, [c_int32, POINTER(RpaCell), POINTER(c_int32), c_int32, PD, PD, PPD,
                             PPD, PPD, POINTER(RpaOptions), PD, PD, POINTER(c_int32),
                             POINTER(RpaStats), c_void_p, c_size_t, c_void_p]),
    "rpa_energy_backward": (c_int32, [POINTER(RpaCell), c_int32, PD, PD, c_int32, c_void_p,
                                      c_void_p, c_double, c_void_p, POINTER(RpaOptions),
                                      POINTER(RpaStats), c_void_p, c_size_t, c_void_p]),
}

_lib = None


def load(path=None):
    """Load the shared library once; raises OSError if it has not been built."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise OSError("librpa_gfx950.so not found at %s: build it first (python -m paper_2504_01816_amd.build)" % p)
    lib = ctypes.CDLL(p)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = lib
    return lib


def default_options(**kw):
    o = RpaOptions()
    rc = load().rpa_default_options(ctypes.byref(o))
    if rc != 0:
        raise RuntimeError("rpa_default_options failed")
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def last_error():
    return load().rpa_last_error().decode()


def check(rc, what):
    if rc < 0:
        raise RuntimeError("%s failed: %s (%s)" % (what, load().rpa_error_string(rc).decode(),
                                                   last_error()))
    return rc
