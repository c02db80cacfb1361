"""Differentiable homogenization: torch.autograd.Function over the HIP forward
path and its hand-written adjoint (Eq. (9)).

``Homogenize.apply(pos, q, spec)`` maps charge positions (B, N, 3) and values
(B, N) (float64, any device; they are read on the host) to C^H (B, 6, 6) and
V (B,) on the CPU.  ``spec`` fixes everything else: resolution, spectral
weights, the logistic sharpness kappa and the half-thickness t of each design
(held fixed -- set it once from a target volume with ``initial_thickness``),
materials and solver options.  The backward pass calls the library's adjoint
with the workspaces the forward kept: no second solve.
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
    thickness: List[float]
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
    state: dict = dc_field(default_factory=dict)

    def designs(self, pos, q):
        out = []
        for b in range(pos.shape[0]):
            out.append(Design(pos=pos[b], q=q[b], n=self.n, K=self.K, alpha=self.alpha, iso=self.iso,
                              thickness=float(self.thickness[b]), kappa=self.kappa, dist_mode=self.dist_mode,
                              E=self.E, nu=self.nu, E_void=self.E_void))
        return out


def initial_thickness(designs):
    """Half-thickness of each design for its target volume (field step only)."""
    return [api.field(d)["t"] for d in designs]


class Homogenize(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos, q, spec):
        if spec.kappa <= 0:
            raise ValueError("gradients need the logistic occupancy (kappa > 0)")
        P = pos.detach().to("cpu", torch.float64).numpy()
        Q = q.detach().to("cpu", torch.float64).numpy()
        designs = spec.designs(P, Q)
        outs, ws, opts = api.homogenize_batch(designs, precision=spec.precision, rtol=spec.rtol,
                                              max_iter=spec.max_iter, save_for_backward=True,
                                              return_workspaces=True, solver=spec.solver)
        spec.state["last"] = outs
        ctx.spec = spec
        ctx.designs = designs
        ctx.ws = ws
        ctx.opts = opts
        ctx.pos_meta = (pos.device, pos.dtype)
        ctx.q_meta = (q.device, q.dtype)
        C = torch.tensor(np.stack([o["C"] for o in outs]), dtype=torch.float64)
        V = torch.tensor([o["V"] for o in outs], dtype=torch.float64)
        return C, V

    @staticmethod
    def backward(ctx, gC, gV):
        Bsz = len(ctx.designs)
        gC = torch.zeros((Bsz, 6, 6), dtype=torch.float64) if gC is None else gC.detach().cpu().double()
        gV = torch.zeros(Bsz, dtype=torch.float64) if gV is None else gV.detach().cpu().double()
        gpos, gq = [], []
        for b, d in enumerate(ctx.designs):
            dp, dq = api.grad(d, ctx.opts, ctx.ws[b], gC[b].numpy(), float(gV[b]))
            gpos.append(dp)
            gq.append(dq)
        gpos = torch.tensor(np.stack(gpos), dtype=ctx.pos_meta[1], device=ctx.pos_meta[0])
        gq = torch.tensor(np.stack(gq), dtype=ctx.q_meta[1], device=ctx.q_meta[0])
        return gpos, gq, None


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
