"""ctypes binding of libshellhom (include/shellhom.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  PyTorch provides device memory (workspaces, arenas, input/output
tensors) and the current HIP stream.  The library must be built in-tree
(``python -m paper_2511_04025_amd.build``); loading fails loudly otherwise --
there is no CPU fallback.
"""
import ctypes
import os
from ctypes import POINTER, c_double, c_int32, c_size_t, c_uint64, c_void_p

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# SHH_LIB_PATH selects another build of the same library (A/B timing of kernel
# variants); the default is the in-tree build.
LIB_PATH = os.environ.get("SHH_LIB_PATH") or os.path.join(HERE, "libshellhom.so")

SHH_OK = 0
SHH_NOT_CONVERGED = 1
SHH_INVALID_ARG = -1
SHH_WORKSPACE_TOO_SMALL = -2
SHH_HIP_ERROR = -3
SHH_OVER_BUDGET = -4
SHH_UNSUPPORTED = -5
SHH_BREAKDOWN = -6
SHH_NOT_FOUND = -7
SHH_SCRATCH_TOO_SMALL = -8
NOALLOC_SCRATCH_BYTES = 128 << 20

PREC_FP64 = 0
PREC_MIXED = 1


class ShhDesign(ctypes.Structure):
    _fields_ = [
        ("n", c_int32), ("num_charges", c_int32),
        ("pos", POINTER(c_double)), ("q", POINTER(c_double)),
        ("K", c_int32), ("alpha", POINTER(c_double)),
        ("iso", c_double), ("thickness", c_double), ("target_vf", c_double), ("kappa", c_double),
        ("dist_mode", c_int32),
        ("E", c_double), ("nu", c_double), ("E_void", c_double),
        ("symmetry", c_int32),
    ]


class ShhOpts(ctypes.Structure):
    _fields_ = [
        ("precision", c_int32), ("rtol", c_double), ("max_iter", c_int32),
        ("recompute_every", c_int32), ("save_for_backward", c_int32), ("check_every", c_int32),
        ("solver", c_int32),
    ]


class ShhResult(ctypes.Structure):
    _fields_ = [
        ("CH", c_double * 36), ("vol_frac", c_double), ("t_used", c_double),
        ("iters", c_int32 * 6), ("rel_res", c_double * 6), ("ms", c_double * 5), ("status", c_int32),
        ("active_nodes", c_int32),
    ]


EXPORTS = {
    "shh_version": (c_int32, []),
    "shh_strerror": (ctypes.c_char_p, [c_int32]),
    "shh_workspace_bytes": (c_int32, [POINTER(ShhDesign), POINTER(ShhOpts), POINTER(c_size_t)]),
    "shh_homogenize": (c_int32, [POINTER(ShhDesign), POINTER(ShhOpts), c_void_p, c_size_t, c_void_p,
                                 POINTER(ShhResult)]),
    "shh_homogenize_noalloc": (c_int32, [POINTER(ShhDesign), POINTER(ShhOpts), c_void_p, POINTER(ShhResult)]),
    "shh_homogenize_batch": (c_int32, [POINTER(ShhDesign), c_int32, POINTER(ShhOpts), POINTER(c_void_p),
                                       POINTER(c_size_t), c_void_p, POINTER(ShhResult)]),
    "shh_workspace_bytes_stiffness": (c_int32, [c_int32, POINTER(ShhOpts), POINTER(c_size_t)]),
    "shh_workspace_bytes_operator": (c_int32, [c_int32, c_int32, POINTER(c_size_t)]),
    "shh_mg_operator": (c_int32, [c_int32, c_int32, c_void_p, c_double, c_int32, c_void_p, c_void_p, c_void_p,
                                  c_size_t, c_void_p]),
    "shh_homogenize_stiffness": (c_int32, [c_int32, c_void_p, c_double, POINTER(ShhOpts), c_void_p, c_size_t,
                                           c_void_p, POINTER(ShhResult)]),
    "shh_homogenize_field": (c_int32, [c_int32, c_void_p, c_int32, c_double, c_double, c_double,
                                       POINTER(ShhOpts), c_void_p, c_size_t, c_void_p, POINTER(ShhResult)]),
    "shh_field": (c_int32, [POINTER(ShhDesign), c_void_p, c_size_t, c_void_p, c_void_p, c_void_p, c_void_p,
                            c_void_p, POINTER(ShhResult)]),
    "shh_workspace_bytes_points": (c_int32, [POINTER(ShhDesign), c_int32, POINTER(c_size_t)]),
    "shh_field_points": (c_int32, [POINTER(ShhDesign), c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t,
                                   c_void_p]),
    "shh_field_points_grad": (c_int32, [POINTER(ShhDesign), c_int32, c_void_p, c_void_p, POINTER(c_double),
                                        POINTER(c_double), POINTER(c_double), c_void_p, c_size_t, c_void_p]),
    "shh_apply_stiffness": (c_int32, [c_int32, c_int32, c_void_p, c_double, c_int32, c_void_p, c_void_p,
                                      c_void_p, c_size_t, c_void_p]),
    "shh_load_vectors": (c_int32, [c_int32, c_void_p, c_double, c_void_p, c_void_p, c_size_t, c_void_p]),
    "shh_energy": (c_int32, [c_int32, c_void_p, c_double, c_void_p, POINTER(c_double), c_void_p, c_size_t,
                             c_void_p]),
    "shh_grad": (c_int32, [POINTER(ShhDesign), POINTER(ShhOpts), c_void_p, c_size_t, POINTER(c_double),
                           c_double, POINTER(c_double), POINTER(c_double), POINTER(c_double),
                           POINTER(c_double), c_void_p]),
    "shh_grad_batch": (c_int32, [POINTER(ShhDesign), c_int32, POINTER(ShhOpts), POINTER(c_void_p),
                                 POINTER(c_size_t), POINTER(c_double), POINTER(c_double), POINTER(c_double),
                                 POINTER(c_double), POINTER(c_double), POINTER(c_double), c_void_p]),
    "shh_profile_enable": (c_int32, [c_int32]),
    "shh_profile_read": (c_int32, [c_int32, POINTER(ctypes.c_int64), POINTER(c_double)]),
    "shh_stream_copy": (c_int32, [c_void_p, c_void_p, c_size_t, c_void_p]),
    "shh_engine_create": (c_int32, [c_void_p, c_size_t, c_int32, c_void_p, POINTER(c_void_p)]),
    "shh_engine_footprint": (c_int32, [POINTER(ShhDesign), POINTER(ShhOpts), POINTER(c_size_t)]),
    "shh_engine_submit": (c_int32, [c_void_p, POINTER(ShhDesign), POINTER(ShhOpts), c_uint64]),
    "shh_engine_step": (c_int32, [c_void_p, c_int32, POINTER(c_int32), POINTER(c_int32)]),
    "shh_engine_poll": (c_int32, [c_void_p, POINTER(ShhResult), POINTER(c_uint64), c_int32, POINTER(c_int32)]),
    "shh_engine_cancel": (c_int32, [c_void_p, c_uint64]),
    "shh_engine_destroy": (None, [c_void_p]),
}

_LIB = None


class ShellhomError(RuntimeError):
    def __init__(self, code, where=""):
        self.code = code
        msg = lib().shh_strerror(code).decode() if _LIB is not None else str(code)
        super().__init__(f"{where}: {msg} (status {code})")


def lib():
    """Load libshellhom.so (built in-tree); raises if it is missing."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2511_04025_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def check(code, where):
    if code < 0:
        raise ShellhomError(code, where)
    return code


def _dptr(a):
    return a.ctypes.data_as(POINTER(c_double))


class DesignArgs:
    """Keeps the NumPy buffers alive while a ShhDesign points into them."""

    def __init__(self, design):
        self.pos = np.ascontiguousarray(np.asarray(design.pos, dtype=np.float64).reshape(-1, 3))
        self.q = np.ascontiguousarray(np.asarray(design.q, dtype=np.float64).ravel())
        self.alpha = None if design.alpha is None else np.ascontiguousarray(
            np.asarray(design.alpha, dtype=np.float64).ravel())
        th = design.thickness
        self.c = ShhDesign(
            n=int(design.n), num_charges=int(self.q.size), pos=_dptr(self.pos), q=_dptr(self.q),
            K=int(design.K), alpha=_dptr(self.alpha) if self.alpha is not None else None,
            iso=float(design.iso), thickness=-1.0 if th is None else float(th),
            target_vf=0.0 if design.target_vf is None else float(design.target_vf),
            kappa=float(design.kappa), dist_mode=int(design.dist_mode),
            E=float(design.E), nu=float(design.nu), E_void=float(design.E_void),
            symmetry=SYMMETRY[getattr(design, "symmetry", 0)])


SOLVER_JACOBI, SOLVER_MG, SOLVER_AUTO, SOLVER_SELECTIVE, SOLVER_SELECTIVE_JACOBI = 0, 1, 2, 3, 4
# fundamental bounding volumes (Sec. 3.2): by name or by the C constant
SYMMETRY = {0: 0, 1: 1, 2: 2, None: 0, "none": 0, "mirror": 1, "cubic": 2}
PROF_KINDS = ("cg_pass", "mg_dir", "mg_step1", "mg_res", "mg_post", "mg_last", "mg_update", "mg_restrict",
              "mg_prolong", "mg_apply1", "resid64", "sel_op", "sel_update", "sel_resid", "sel_mg_pq",
              "sel_mg_smooth", "sel_mg_vec", "sel_mg_transfer")
EDTYPE_U8, EDTYPE_F32, EDTYPE_F64 = 0, 1, 2


def make_opts(precision="mixed", rtol=None, max_iter=20000, recompute_every=0, save_for_backward=False,
              check_every=0, solver="jacobi"):
    prec = PREC_MIXED if precision in ("mixed", PREC_MIXED) else PREC_FP64
    if rtol is None:
        rtol = 1e-6 if prec == PREC_MIXED else 1e-10
    sv = {"mg": SOLVER_MG, "jacobi": SOLVER_JACOBI, "auto": SOLVER_AUTO,
          "selective": SOLVER_SELECTIVE, "selective-jacobi": SOLVER_SELECTIVE_JACOBI}.get(solver, solver)
    if sv not in (SOLVER_MG, SOLVER_JACOBI, SOLVER_AUTO, SOLVER_SELECTIVE, SOLVER_SELECTIVE_JACOBI):
        raise ValueError(f"unknown solver {solver!r}")
    return ShhOpts(precision=prec, rtol=float(rtol), max_iter=int(max_iter),
                   recompute_every=int(recompute_every), save_for_backward=int(bool(save_for_backward)),
                   check_every=int(check_every), solver=sv)


def result_dict(r):
    return {
        "C": np.array(r.CH[:], dtype=np.float64).reshape(6, 6),
        "V": float(r.vol_frac),
        "t": float(r.t_used),
        "iters": np.array(r.iters[:], dtype=np.int64),
        "rel_res": np.array(r.rel_res[:], dtype=np.float64),
        "ms": {k: float(v) for k, v in zip(("field", "rhs", "solve", "C", "all"), r.ms[:])},
        "status": int(r.status),
        "active_nodes": int(r.active_nodes),
    }
