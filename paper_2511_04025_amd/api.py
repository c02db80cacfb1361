"""Python entry points over libshellhom (same names as the C ABI, minus the
shh_ prefix).  PyTorch supplies device memory and the current HIP stream; all
arithmetic of the path runs in the library's HIP kernels.

Layouts: voxel grids are tensors of shape (n, n, n) indexed [k, j, i] (x
fastest); six-load-case nodal fields are (6, 3, n, n, n); C^H is 6x6 in Voigt
order (11, 22, 33, 23, 13, 12) with engineering shear.
"""
import ctypes
from ctypes import byref, c_double, c_size_t, c_void_p

import numpy as np
import torch

from . import binding as B


def _require_gpu():
    if not torch.cuda.is_available():
        raise RuntimeError("libshellhom needs a HIP GPU (torch.cuda.is_available() is False)")


def _stream():
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return c_void_p(t.data_ptr())


def _alloc(nbytes):
    return torch.empty(int(nbytes) + 256, dtype=torch.uint8, device="cuda")


class Workspace:
    """Device workspace of one design (a torch uint8 tensor)."""

    def __init__(self, nbytes):
        self.tensor = _alloc(nbytes)
        self.nbytes = self.tensor.numel()

    @property
    def ptr(self):
        return _ptr(self.tensor)


def workspace_bytes(design, opts):
    a = B.DesignArgs(design)
    nb = c_size_t(0)
    B.check(B.lib().shh_workspace_bytes(byref(a.c), byref(opts), byref(nb)), "shh_workspace_bytes")
    return nb.value


def homogenize(design, precision="mixed", rtol=None, max_iter=20000, recompute_every=0,
               save_for_backward=False, check_every=0, workspace=None, return_workspace=False, solver="jacobi"):
    """The whole path for one design; returns a dict with C (6x6), V, t,
    iters, rel_res, ms, status (and the workspace if asked)."""
    _require_gpu()
    opts = B.make_opts(precision, rtol, max_iter, recompute_every, save_for_backward, check_every, solver)
    a = B.DesignArgs(design)
    need = workspace_bytes(design, opts)
    if workspace is None or workspace.nbytes < need:
        workspace = Workspace(need)
    res = B.ShhResult()
    rc = B.lib().shh_homogenize(byref(a.c), byref(opts), workspace.ptr, c_size_t(workspace.nbytes),
                                _stream(), byref(res))
    B.check(rc, "shh_homogenize")
    out = B.result_dict(res)
    if return_workspace:
        out["workspace"] = workspace
        out["opts"] = opts
    return out


def homogenize_noalloc(design, precision="mixed", rtol=None, max_iter=20000, recompute_every=0,
                       check_every=0, solver="jacobi"):
    """shh_homogenize_noalloc: the path on the library's fixed device scratch
    (no workspace, no device allocation by the call); same result dict as
    homogenize (ms all zero).  Raises for designs larger than the scratch."""
    _require_gpu()
    opts = B.make_opts(precision, rtol, max_iter, recompute_every, False, check_every, solver)
    a = B.DesignArgs(design)
    res = B.ShhResult()
    B.check(B.lib().shh_homogenize_noalloc(byref(a.c), byref(opts), _stream(), byref(res)),
            "shh_homogenize_noalloc")
    return B.result_dict(res)


def homogenize_batch(designs, precision="mixed", rtol=None, max_iter=20000, recompute_every=0,
                     save_for_backward=False, check_every=0, workspaces=None, return_workspaces=False,
                     solver="jacobi"):
    """All designs at once, one batched launch per phase."""
    _require_gpu()
    opts = B.make_opts(precision, rtol, max_iter, recompute_every, save_for_backward, check_every, solver)
    args = [B.DesignArgs(d) for d in designs]
    count = len(designs)
    arr = (B.ShhDesign * count)(*[a.c for a in args])
    if workspaces is None:
        workspaces = [Workspace(workspace_bytes(d, opts)) for d in designs]
    ptrs = (c_void_p * count)(*[w.ptr.value for w in workspaces])
    sizes = (c_size_t * count)(*[w.nbytes for w in workspaces])
    res = (B.ShhResult * count)()
    rc = B.lib().shh_homogenize_batch(arr, count, byref(opts), ptrs, sizes, _stream(), res)
    B.check(rc, "shh_homogenize_batch")
    outs = [B.result_dict(r) for r in res]
    if return_workspaces:
        return outs, workspaces, opts
    return outs


def stiffness_workspace_bytes(n, precision="fp64", solver="jacobi"):
    opts = B.make_opts(precision, solver=solver)
    nb = c_size_t(0)
    B.check(B.lib().shh_workspace_bytes_stiffness(int(n), byref(opts), byref(nb)), "shh_workspace_bytes_stiffness")
    return nb.value


def operator_workspace_bytes(n, precision="fp64"):
    """Device bytes the operator calls (apply_stiffness, load_vectors, energy) need."""
    prec = B.PREC_FP64 if precision == "fp64" else B.PREC_MIXED
    nb = c_size_t(0)
    B.check(B.lib().shh_workspace_bytes_operator(int(n), prec, byref(nb)), "shh_workspace_bytes_operator")
    return nb.value


def _check_grid(E):
    if not (E.is_cuda and E.dtype == torch.float64 and E.dim() == 3 and E.is_contiguous()
            and E.shape[0] == E.shape[1] == E.shape[2]):
        raise ValueError("E must be a contiguous float64 CUDA tensor of shape (n, n, n)")
    return E.shape[0]


def homogenize_stiffness(E, nu, precision="mixed", rtol=None, max_iter=20000, recompute_every=0,
                         check_every=0, solver="jacobi"):
    """Steps 3-4 for a given voxel modulus field E (n, n, n) float64 on the GPU."""
    _require_gpu()
    n = _check_grid(E)
    opts = B.make_opts(precision, rtol, max_iter, recompute_every, False, check_every, solver)
    nb = c_size_t(0)
    B.check(B.lib().shh_workspace_bytes_stiffness(n, byref(opts), byref(nb)), "shh_workspace_bytes_stiffness")
    ws = Workspace(nb.value)
    res = B.ShhResult()
    rc = B.lib().shh_homogenize_stiffness(n, _ptr(E), c_double(nu), byref(opts), ws.ptr, c_size_t(ws.nbytes),
                                          _stream(), byref(res))
    B.check(rc, "shh_homogenize_stiffness")
    return B.result_dict(res)


def homogenize_field(E, nu, E_solid=1.0, E_void=0.0, precision="mixed", rtol=None, max_iter=20000,
                     recompute_every=0, check_every=0, solver="jacobi"):
    """Steps 3-4 for a voxel grid E (n, n, n) on the GPU in one of three
    encodings, chosen by its dtype: uint8 (solid/void code: E_solid where
    nonzero, E_void where zero), float32 or float64 moduli."""
    _require_gpu()
    codes = {torch.uint8: B.EDTYPE_U8, torch.float32: B.EDTYPE_F32, torch.float64: B.EDTYPE_F64}
    if not (E.is_cuda and E.dtype in codes and E.dim() == 3 and E.is_contiguous()
            and E.shape[0] == E.shape[1] == E.shape[2]):
        raise ValueError("E must be a contiguous uint8/float32/float64 CUDA tensor of shape (n, n, n)")
    n = E.shape[0]
    opts = B.make_opts(precision, rtol, max_iter, recompute_every, False, check_every, solver)
    nb = c_size_t(0)
    B.check(B.lib().shh_workspace_bytes_stiffness(n, byref(opts), byref(nb)), "shh_workspace_bytes_stiffness")
    ws = Workspace(nb.value)
    res = B.ShhResult()
    rc = B.lib().shh_homogenize_field(n, _ptr(E), codes[E.dtype], c_double(E_solid), c_double(E_void),
                                      c_double(nu), byref(opts), ws.ptr, c_size_t(ws.nbytes), _stream(),
                                      byref(res))
    B.check(rc, "shh_homogenize_field")
    return B.result_dict(res)


def field(design):
    """Steps 1-2: F (n,n,n), G (3,n,n,n), d (n,n,n), beta (n,n,n) as float64 CUDA
    tensors, plus V and t."""
    _require_gpu()
    n = int(design.n)
    opts = B.make_opts("fp64")
    ws = Workspace(workspace_bytes(design, opts))
    F = torch.empty((n, n, n), dtype=torch.float64, device="cuda")
    G = torch.empty((3, n, n, n), dtype=torch.float64, device="cuda")
    d = torch.empty((n, n, n), dtype=torch.float64, device="cuda")
    beta = torch.empty((n, n, n), dtype=torch.float64, device="cuda")
    a = B.DesignArgs(design)
    res = B.ShhResult()
    rc = B.lib().shh_field(byref(a.c), ws.ptr, c_size_t(ws.nbytes), _ptr(F), _ptr(G), _ptr(d), _ptr(beta),
                           _stream(), byref(res))
    B.check(rc, "shh_field")
    return {"F": F, "G": G, "d": d, "beta": beta, "V": float(res.vol_frac), "t": float(res.t_used)}


def apply_stiffness(E, p, nu, precision="fp64"):
    """q = K p for nodal fields p (m, 3, n, n, n), m <= 6 (float64 for 'fp64',
    float32 for 'mixed')."""
    _require_gpu()
    n = _check_grid(E)
    want = torch.float64 if precision == "fp64" else torch.float32
    if not (p.is_cuda and p.dtype == want and p.is_contiguous() and p.shape[1:] == (3, n, n, n)):
        raise ValueError("p must be a contiguous CUDA tensor (m, 3, n, n, n) of the precision's dtype")
    m = p.shape[0]
    q = torch.empty_like(p)
    ws = Workspace(operator_workspace_bytes(n, precision))
    prec = B.PREC_FP64 if precision == "fp64" else B.PREC_MIXED
    rc = B.lib().shh_apply_stiffness(n, prec, _ptr(E), c_double(nu), m, _ptr(p), _ptr(q), ws.ptr,
                                     c_size_t(ws.nbytes), _stream())
    B.check(rc, "shh_apply_stiffness")
    return q


def mg_operator(E, v, nu, level, precision="fp64"):
    """q = A_level v for the multigrid hierarchy's Galerkin operator of level
    `level` >= 1; v (6, 3, m, m, m) with m = n / 2^level."""
    _require_gpu()
    n = _check_grid(E)
    want = torch.float64 if precision == "fp64" else torch.float32
    m = n >> level
    if not (v.is_cuda and v.dtype == want and v.is_contiguous() and tuple(v.shape) == (6, 3, m, m, m)):
        raise ValueError("v must be a contiguous CUDA tensor (6, 3, m, m, m) of the precision's dtype")
    q = torch.empty_like(v)
    ws = Workspace(stiffness_workspace_bytes(n, precision, solver="mg"))
    prec = B.PREC_FP64 if precision == "fp64" else B.PREC_MIXED
    rc = B.lib().shh_mg_operator(n, prec, _ptr(E), c_double(nu), int(level), _ptr(v), _ptr(q), ws.ptr,
                                 c_size_t(ws.nbytes), _stream())
    B.check(rc, "shh_mg_operator")
    return q


def load_vectors(E, nu):
    """f^(k) of the six load cases, (6, 3, n, n, n) float64."""
    _require_gpu()
    n = _check_grid(E)
    f = torch.empty((6, 3, n, n, n), dtype=torch.float64, device="cuda")
    ws = Workspace(operator_workspace_bytes(n, "fp64"))
    rc = B.lib().shh_load_vectors(n, _ptr(E), c_double(nu), _ptr(f), ws.ptr, c_size_t(ws.nbytes), _stream())
    B.check(rc, "shh_load_vectors")
    return f


def energy(E, u, nu):
    """Energy form of C^H for displacements u (6, 3, n, n, n) float64."""
    _require_gpu()
    n = _check_grid(E)
    if not (u.is_cuda and u.dtype == torch.float64 and u.is_contiguous() and u.shape == (6, 3, n, n, n)):
        raise ValueError("u must be a contiguous float64 CUDA tensor (6, 3, n, n, n)")
    ws = Workspace(operator_workspace_bytes(n, "fp64"))
    C = (c_double * 36)()
    rc = B.lib().shh_energy(n, _ptr(E), c_double(nu), _ptr(u), C, ws.ptr, c_size_t(ws.nbytes), _stream())
    B.check(rc, "shh_energy")
    return np.array(C[:]).reshape(6, 6)


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(c_double))


def grad(design, opts, workspace, dL_dC, dL_dV, full=False):
    """Adjoint of a forward run with save_for_backward: (dL/dpos (N,3), dL/dq (N,)),
    and with full=True also dL/dalpha ((K+1)^3,) and dL/dt (t held free)."""
    _require_gpu()
    a = B.DesignArgs(design)
    N = a.q.size
    K1 = int(design.K) + 1
    g = np.ascontiguousarray(np.asarray(dL_dC, dtype=np.float64).reshape(36))
    dpos = np.zeros((N, 3))
    dq = np.zeros(N)
    dalpha = np.zeros(K1 ** 3)
    dt = np.zeros(1)
    rc = B.lib().shh_grad(byref(a.c), byref(opts), workspace.ptr, c_size_t(workspace.nbytes), _dp(g),
                          c_double(float(dL_dV)), _dp(dpos), _dp(dq), _dp(dalpha), _dp(dt), _stream())
    B.check(rc, "shh_grad")
    if full:
        return dpos, dq, dalpha.reshape(K1, K1, K1), float(dt[0])
    return dpos, dq


def grad_batch(designs, opts, workspaces, dL_dC, dL_dV):
    """Adjoint of one homogenize_batch call (one synchronization for all
    designs): lists of dL/dpos (N_i,3), dL/dq (N_i,), dL/dalpha ((K_i+1)^3 as
    (K+1,K+1,K+1)) and an array of dL/dt."""
    _require_gpu()
    args = [B.DesignArgs(d) for d in designs]
    count = len(designs)
    arr = (B.ShhDesign * count)(*[a.c for a in args])
    ptrs = (c_void_p * count)(*[w.ptr.value for w in workspaces])
    sizes = (c_size_t * count)(*[w.nbytes for w in workspaces])
    gC = np.ascontiguousarray(np.asarray(dL_dC, dtype=np.float64).reshape(count, 36))
    gV = np.ascontiguousarray(np.asarray(dL_dV, dtype=np.float64).reshape(count))
    Ns = [a.q.size for a in args]
    K1s = [int(d.K) + 1 for d in designs]
    dpos = np.zeros((sum(Ns), 3))
    dq = np.zeros(sum(Ns))
    dalpha = np.zeros(sum(k ** 3 for k in K1s))
    dt = np.zeros(count)
    rc = B.lib().shh_grad_batch(arr, count, byref(opts), ptrs, sizes, _dp(gC), _dp(gV), _dp(dpos), _dp(dq),
                                _dp(dalpha), _dp(dt), _stream())
    B.check(rc, "shh_grad_batch")
    out_p, out_q, out_a = [], [], []
    o = oa = 0
    for N, K1 in zip(Ns, K1s):
        out_p.append(dpos[o:o + N])
        out_q.append(dq[o:o + N])
        out_a.append(dalpha[oa:oa + K1 ** 3].reshape(K1, K1, K1))
        o += N
        oa += K1 ** 3
    return out_p, out_q, out_a, dt


def _points(pts):
    pts = torch.as_tensor(pts, dtype=torch.float64)
    if pts.dim() != 2 or pts.shape[1] != 3:
        raise ValueError("points must be (M, 3)")
    return pts.to("cuda").contiguous()


def _points_workspace(a, npts):
    nb = c_size_t(0)
    B.check(B.lib().shh_workspace_bytes_points(byref(a.c), int(npts), byref(nb)), "shh_workspace_bytes_points")
    return Workspace(nb.value)


def field_points(design, pts, gradient=False):
    """F of Eq. (6) at arbitrary points (M, 3) -> (M,) float64 CUDA tensor (and
    its gradient (3, M) if asked); only the design's charges, alpha, K and
    symmetry are used."""
    _require_gpu()
    a = B.DesignArgs(design)
    P = _points(pts)
    M = P.shape[0]
    ws = _points_workspace(a, M)
    F = torch.empty(M, dtype=torch.float64, device="cuda")
    G = torch.empty((3, M), dtype=torch.float64, device="cuda") if gradient else None
    B.check(B.lib().shh_field_points(byref(a.c), M, _ptr(P), _ptr(F), _ptr(G) if G is not None else None, ws.ptr,
                                     c_size_t(ws.nbytes), _stream()), "shh_field_points")
    return (F, G) if gradient else F


def field_points_grad(design, pts, dL_dF):
    """Adjoint of field_points: dL/dpos (N, 3), dL/dq (N,), dL/dalpha (K+1,)*3."""
    _require_gpu()
    a = B.DesignArgs(design)
    P = _points(pts)
    M = P.shape[0]
    g = torch.as_tensor(dL_dF, dtype=torch.float64).to("cuda").contiguous()
    ws = _points_workspace(a, M)
    N = a.q.size
    K1 = int(design.K) + 1
    dpos, dq, dal = np.zeros((N, 3)), np.zeros(N), np.zeros(K1 ** 3)
    B.check(B.lib().shh_field_points_grad(byref(a.c), M, _ptr(P), _ptr(g), _dp(dpos), _dp(dq), _dp(dal), ws.ptr,
                                          c_size_t(ws.nbytes), _stream()), "shh_field_points_grad")
    return dpos, dq, dal.reshape(K1, K1, K1)
