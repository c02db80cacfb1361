"""Differentiable homogenization: torch.autograd.Function over the HIP forward
path and its hand-written adjoint (Eq. (9)).

``Homogenize.apply(pos, q, spec, alpha=None, thickness=None)`` maps charge
positions (B, N, 3) and values (B, N) -- and optionally the spectral weights
alpha ((K+1,)*3 shared by the batch, or (B, K+1, K+1, K+1)) and the
half-thicknesses t (B,) -- to C^H (B, 6, 6) and V (B,) on the CPU (inputs are
float64 on any device and are read on the host).  ``spec`` fixes everything
else: resolution, the logistic sharpness kappa, materials, solver options, and
how t is set:

* ``spec.target_vf`` None: t comes from the ``thickness`` input if given, else
  from ``spec.thickness`` (fixed numbers, e.g. ``initial_thickness``); t is a
  free parameter and receives dL/dt.
* ``spec.target_vf`` set: every forward chooses t by bisection so that V
  equals the target (Sec. 4.3's volume constraint), and the backward returns
  the gradient along that constraint (implicit function theorem: dt/dtheta =
  -(dV/dtheta)/(dV/dt)), from a second adjoint of V on the same workspaces.

The backward pass calls the library's batched adjoint with the workspaces the
forward kept: no second solve.
"""
from dataclasses import dataclass, field as dc_field
from typing import List, Optional

import numpy as np
import torch

from . import api
from . import binding as B
from .workloads import Design


@dataclass
class Spec:
    n: int
    thickness: Optional[List[float]]
    kappa: float
    K: int = 3
    alpha: Optional[np.ndarray] = None
    iso: float = 0.0
    dist_mode: int = 0
    E: float = 1.0
    nu: float = 0.3
    E_void: float = 1e-6
    precision: str = "mixed"
    rtol: Optional[float] = None
    max_iter: int = 20000
    solver: str = "jacobi"
    target_vf: Optional[float] = None
    symmetry: object = 0  # fundamental bounding volume of the charges (workloads.Design.symmetry)
    state: dict = dc_field(default_factory=dict)

    def designs(self, pos, q, alpha=None, thickness=None):
        out = []
        for b in range(pos.shape[0]):
            if alpha is None:
                al = self.alpha
            else:
                al = alpha if alpha.ndim == 3 else alpha[b]
            if self.target_vf is not None:
                th, vf = None, float(self.target_vf)
            else:
                th = float(thickness[b]) if thickness is not None else float(self.thickness[b])
                vf = None
            out.append(Design(pos=pos[b], q=q[b], n=self.n, K=self.K, alpha=al, iso=self.iso,
                              thickness=th, target_vf=vf, kappa=self.kappa, dist_mode=self.dist_mode,
                              E=self.E, nu=self.nu, E_void=self.E_void, symmetry=self.symmetry))
        return out


def initial_thickness(designs):
    """Half-thickness of each design for its target volume (field step only)."""
    return [api.field(d)["t"] for d in designs]


def _host(x):
    return None if x is None else x.detach().to("cpu", torch.float64).numpy()


def _like(arr, ref):
    return torch.tensor(arr, dtype=ref.dtype, device=ref.device)


class Homogenize(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos, q, spec, alpha=None, thickness=None):
        if spec.kappa <= 0:
            raise ValueError("gradients need the logistic occupancy (kappa > 0)")
        if thickness is not None and spec.target_vf is not None:
            raise ValueError("thickness is set by the volume constraint when spec.target_vf is given")
        designs = spec.designs(_host(pos), _host(q), _host(alpha), _host(thickness))
        outs, ws, opts = api.homogenize_batch(designs, precision=spec.precision, rtol=spec.rtol,
                                              max_iter=spec.max_iter, save_for_backward=True,
                                              return_workspaces=True, solver=spec.solver)
        spec.state["last"] = outs
        ctx.spec = spec
        # the adjoint evaluates at the forward's own t (given or bisected)
        ctx.designs = [d.with_(thickness=o["t"], target_vf=None) for d, o in zip(designs, outs)]
        ctx.ws = ws
        ctx.opts = opts
        ctx.refs = (pos, q, alpha, thickness)
        C = torch.tensor(np.stack([o["C"] for o in outs]), dtype=torch.float64)
        V = torch.tensor([o["V"] for o in outs], dtype=torch.float64)
        return C, V

    @staticmethod
    def backward(ctx, gC, gV):
        Bsz = len(ctx.designs)
        gC = torch.zeros((Bsz, 6, 6), dtype=torch.float64) if gC is None else gC.detach().cpu().double()
        gV = torch.zeros(Bsz, dtype=torch.float64) if gV is None else gV.detach().cpu().double()
        gp, gq, ga, gt = api.grad_batch(ctx.designs, ctx.opts, ctx.ws, gC.numpy(), gV.numpy())
        if ctx.spec.target_vf is not None:
            # along V(theta, t) = V*: subtract (dL/dt / dV/dt) dV/dtheta
            vp, vq, va, vt = api.grad_batch(ctx.designs, ctx.opts, ctx.ws, np.zeros((Bsz, 6, 6)), np.ones(Bsz))
            r = gt / vt
            gp = [a - rb * b for a, b, rb in zip(gp, vp, r)]
            gq = [a - rb * b for a, b, rb in zip(gq, vq, r)]
            ga = [a - rb * b for a, b, rb in zip(ga, va, r)]
            gt = None
        pos, q, alpha, thickness = ctx.refs
        g_pos = _like(np.stack(gp), pos)
        g_q = _like(np.stack(gq), q)
        g_alpha = None
        if alpha is not None:
            A = np.stack(ga)
            g_alpha = _like(A.sum(axis=0) if alpha.dim() == 3 else A, alpha)
        g_t = None if (thickness is None or gt is None) else _like(gt, thickness)
        return g_pos, g_q, None, g_alpha, g_t


def voigt_bulk(C):
    """K_V = (sum of the 3x3 normal block) / 9 for C of shape (..., 6, 6)."""
    return C[..., :3, :3].sum(dim=(-1, -2)) / 9.0


def hill_bulk_shear(C):
    tr_n = C[..., 0, 0] + C[..., 1, 1] + C[..., 2, 2]
    off_n = C[..., :3, :3].sum(dim=(-1, -2)) - tr_n
    tr_s = C[..., 3, 3] + C[..., 4, 4] + C[..., 5, 5]
    KV, GV = (tr_n + off_n) / 9.0, (tr_n - 0.5 * off_n + 3.0 * tr_s) / 15.0
    S = torch.linalg.inv(C)
    str_n = S[..., 0, 0] + S[..., 1, 1] + S[..., 2, 2]
    soff_n = S[..., :3, :3].sum(dim=(-1, -2)) - str_n
    str_s = S[..., 3, 3] + S[..., 4, 4] + S[..., 5, 5]
    KR, GR = 1.0 / (str_n + soff_n), 15.0 / (4.0 * str_n - 2.0 * soff_n + 3.0 * str_s)
    return 0.5 * (KV + KR), 0.5 * (GV + GR)


def bulk_poisson_loss(C, K_target, nu_target=0.0, w_K=1.0, w_nu=1.0):
    """Weighted bulk-modulus / Poisson-ratio objective, summed over the batch:
    w_K (K_V / K* - 1)^2 + w_nu (nu_H - nu*)^2 with nu_H = (3K - 2G) / (2 (3K + G))
    from Hill's K and G."""
    KV = voigt_bulk(C)
    KH, GH = hill_bulk_shear(C)
    nuH = (3.0 * KH - 2.0 * GH) / (2.0 * (3.0 * KH + GH))
    K_target = torch.as_tensor(K_target, dtype=C.dtype)
    return (w_K * (KV / K_target - 1.0) ** 2 + w_nu * (nuH - nu_target) ** 2).sum()
