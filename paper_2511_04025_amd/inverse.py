"""Inverse design over the charge parametrization (Sec. 4.3, objectives of
Sec. 5.4).

The design variables are the charge positions p_m, the spectral weights
alpha_hkl and the half-thickness t.  Sec. 4.3 alternates three stages:

  (i)   t follows the volume constraint (every forward bisects t on the GPU so
        that V equals the target, ``autograd.Spec.target_vf``);
  (ii)  a fixed number of first-order steps on alpha with the positions held,
        using the adjoint of Eq. (9) along the volume constraint;
  (iii) CMA-ES on the positions with alpha held: each generation's population
        is homogenized in one batched call (one launch per phase for the whole
        population), forward only.

The objectives are the six of Sec. 5.4, functions of C^H (and V) only, written
in torch so that stage (ii) differentiates through them.  CMA-ES follows
Hansen's (mu/mu_w, lambda) strategy with cumulative step-size adaptation and
rank-one plus rank-mu covariance updates (N. Hansen, "The CMA Evolution
Strategy: A Tutorial", 2016), written here from that description.

Host-side control only: every homogenization and gradient runs in the HIP
library through ``api`` and ``autograd``.
"""
from dataclasses import dataclass, field as dc_field
from typing import Callable, List, Optional

import numpy as np
import torch

# ---------------------------------------------------------------------------
# objectives (Sec. 5.4); each maps C (B, 6, 6) and V (B,) to values (B,) to
# be minimized
# ---------------------------------------------------------------------------


def _hill(C):
    """Hill averages of bulk and shear modulus (Voigt and Reuss means), with
    every sum over the full normal block (engineering shear in C)."""
    tr_n = C[..., 0, 0] + C[..., 1, 1] + C[..., 2, 2]
    off_n = C[..., :3, :3].sum(dim=(-1, -2)) - tr_n
    tr_s = C[..., 3, 3] + C[..., 4, 4] + C[..., 5, 5]
    KV = (tr_n + off_n) / 9.0
    GV = (tr_n - 0.5 * off_n + 3.0 * tr_s) / 15.0
    S = torch.linalg.inv(C)
    str_n = S[..., 0, 0] + S[..., 1, 1] + S[..., 2, 2]
    soff_n = S[..., :3, :3].sum(dim=(-1, -2)) - str_n
    str_s = S[..., 3, 3] + S[..., 4, 4] + S[..., 5, 5]
    KR = 1.0 / (str_n + soff_n)
    GR = 15.0 / (4.0 * str_n - 2.0 * soff_n + 3.0 * str_s)
    return 0.5 * (KV + KR), 0.5 * (GV + GR)


def young_x(C):
    """E_x = 1 / (C^-1)_11."""
    return 1.0 / torch.linalg.inv(C)[..., 0, 0]


def obj_largest_ex(C, V):
    return -young_x(C) / V


def obj_largest_cavg(C, V):
    return -(C[..., 0, 0] + C[..., 1, 1] + C[..., 2, 2]) / 3.0 / V


def obj_largest_keff(C, V):
    return -_hill(C)[0] / V


def obj_largest_geff(C, V):
    return -_hill(C)[1] / V


def obj_largest_offdiag(C, V):
    """- sum of |C_ij| over the normal rows and shear columns (normal-shear coupling)."""
    return -C[..., :3, 3:].abs().sum(dim=(-1, -2))


def obj_force_response(k, target):
    """|C_kk - target| for a user-chosen diagonal entry k (0-based Voigt index)."""
    def f(C, V):
        return (C[..., k, k] - target).abs()
    return f


OBJECTIVES = {
    "ex": obj_largest_ex,
    "cavg": obj_largest_cavg,
    "keff": obj_largest_keff,
    "geff": obj_largest_geff,
    "offdiag": obj_largest_offdiag,
}


def objective(name, **kw):
    """Objective by name: 'ex', 'cavg', 'keff', 'geff', 'offdiag', or
    'force' (keyword arguments k and target)."""
    if name == "force":
        return obj_force_response(int(kw["k"]), float(kw["target"]))
    return OBJECTIVES[name]


# ---------------------------------------------------------------------------
# CMA-ES
# ---------------------------------------------------------------------------


class CMAES:
    """(mu/mu_w, lambda)-CMA-ES minimizing over R^dim.

    ask() returns a (popsize, dim) array of candidates; tell(X, f) takes them
    back with their objective values and updates the mean, the step size and
    the covariance.  Deterministic for a given seed."""

    def __init__(self, x0, sigma0, popsize=None, seed=0):
        self.m = np.asarray(x0, dtype=np.float64).ravel().copy()
        self.dim = d = self.m.size
        self.sigma = float(sigma0)
        self.lam = int(popsize) if popsize else 4 + int(3 * np.log(d))
        self.mu = self.lam // 2
        w = np.log(self.mu + 0.5) - np.log(np.arange(1, self.mu + 1))
        self.w = w / w.sum()
        self.mueff = 1.0 / np.sum(self.w ** 2)
        self.cs = (self.mueff + 2.0) / (d + self.mueff + 5.0)
        self.ds = 1.0 + 2.0 * max(0.0, np.sqrt((self.mueff - 1.0) / (d + 1.0)) - 1.0) + self.cs
        self.cc = (4.0 + self.mueff / d) / (d + 4.0 + 2.0 * self.mueff / d)
        self.c1 = 2.0 / ((d + 1.3) ** 2 + self.mueff)
        self.cmu = min(1.0 - self.c1, 2.0 * (self.mueff - 2.0 + 1.0 / self.mueff) / ((d + 2.0) ** 2 + self.mueff))
        self.chi = np.sqrt(d) * (1.0 - 1.0 / (4.0 * d) + 1.0 / (21.0 * d * d))
        self.ps = np.zeros(d)
        self.pc = np.zeros(d)
        self.C = np.eye(d)
        self.B = np.eye(d)
        self.D = np.ones(d)
        self.gen = 0
        self.rng = np.random.default_rng(seed)
        self._Y = None

    def ask(self):
        Z = self.rng.standard_normal((self.lam, self.dim))
        self._Y = (Z * self.D) @ self.B.T          # y = B D z
        return self.m + self.sigma * self._Y

    def tell(self, X, fvals):
        X = np.asarray(X, dtype=np.float64)
        Y = (X - self.m) / self.sigma
        order = np.argsort(np.asarray(fvals, dtype=np.float64), kind="stable")
        Ysel = Y[order[: self.mu]]
        yw = self.w @ Ysel
        self.m = self.m + self.sigma * yw
        # C^-1/2 y_w = B D^-1 B^T y_w
        cinv = self.B @ ((self.B.T @ yw) / self.D)
        self.ps = (1.0 - self.cs) * self.ps + np.sqrt(self.cs * (2.0 - self.cs) * self.mueff) * cinv
        nps = np.linalg.norm(self.ps)
        self.gen += 1
        hs = nps / np.sqrt(1.0 - (1.0 - self.cs) ** (2 * self.gen)) < (1.4 + 2.0 / (self.dim + 1.0)) * self.chi
        self.pc = (1.0 - self.cc) * self.pc + (np.sqrt(self.cc * (2.0 - self.cc) * self.mueff) * yw if hs else 0.0)
        dh = 0.0 if hs else self.cc * (2.0 - self.cc)
        rank_mu = (Ysel * self.w[:, None]).T @ Ysel
        self.C = ((1.0 - self.c1 - self.cmu) * self.C + self.c1 * (np.outer(self.pc, self.pc) + dh * self.C)
                  + self.cmu * rank_mu)
        self.sigma *= np.exp((self.cs / self.ds) * (nps / self.chi - 1.0))
        self.C = 0.5 * (self.C + self.C.T)
        evals, evecs = np.linalg.eigh(self.C)
        self.D = np.sqrt(np.maximum(evals, 1e-300))
        self.B = evecs
        return order[0]


# ---------------------------------------------------------------------------
# the alternating pipeline
# ---------------------------------------------------------------------------


@dataclass
class History:
    values: List[float] = dc_field(default_factory=list)     # best objective after each stage
    stages: List[str] = dc_field(default_factory=list)
    thickness: List[float] = dc_field(default_factory=list)  # t chosen by the volume constraint
    evaluations: int = 0


@dataclass
class InverseResult:
    pos: np.ndarray
    q: np.ndarray
    alpha: np.ndarray
    t: float
    value: float
    C: np.ndarray
    V: float
    history: History


def _spec(n, kappa, target_vf, E_void, precision, rtol, solver, K, symmetry=0):
    from . import autograd as AG
    return AG.Spec(n=n, thickness=None, kappa=kappa, K=K, E_void=E_void, precision=precision, rtol=rtol,
                   solver=solver, target_vf=target_vf, symmetry=symmetry)


def evaluate_population(pos_list, q, alpha, spec, obj):
    """Homogenize several position sets (same charges, alpha, t rule) in one
    batched call; returns (objective values, results)."""
    from . import api
    from .workloads import Design
    designs = [Design(pos=np.mod(p, 1.0), q=q, n=spec.n, K=spec.K, alpha=alpha, thickness=None,
                      target_vf=spec.target_vf, kappa=spec.kappa, E_void=spec.E_void, symmetry=spec.symmetry)
               for p in pos_list]
    out = []
    chunk = 64  # the library's largest batch
    for s in range(0, len(designs), chunk):
        out += api.homogenize_batch(designs[s:s + chunk], precision=spec.precision, rtol=spec.rtol,
                                    solver=spec.solver)
    C = torch.tensor(np.stack([o["C"] for o in out]), dtype=torch.float64)
    V = torch.tensor([o["V"] for o in out], dtype=torch.float64)
    with torch.no_grad():
        vals = obj(C, V).numpy()
    return vals, out


def alternating_optimize(pos0, q, n, obj, *, alpha0=None, K=3, target_vf=0.1, kappa=None, E_void=1e-6,
                         rounds=2, alpha_steps=4, alpha_lr=0.05, cma_generations=3, popsize=None,
                         sigma0=0.03, precision="mixed", rtol=3e-6, solver="auto", seed=0, symmetry=0,
                         callback: Optional[Callable] = None) -> InverseResult:
    """Sec. 4.3's alternating scheme: per round, (i) the volume constraint sets
    t (bisection inside every forward), (ii) `alpha_steps` Adam steps on
    alpha along the constraint, (iii) `cma_generations` CMA-ES generations on
    the positions.  kappa defaults to 4 n (a one-voxel transition).  With a
    symmetry mode the positions are those of the fundamental bounding volume
    (Sec. 3.2): every evaluation mirrors them over the cell."""
    from . import autograd as AG
    kappa = 4.0 * n if kappa is None else float(kappa)
    spec = _spec(n, kappa, target_vf, E_void, precision, rtol, solver, K, symmetry)
    pos = np.mod(np.asarray(pos0, dtype=np.float64).reshape(-1, 3), 1.0)
    q = np.asarray(q, dtype=np.float64).ravel()
    alpha = np.ones((K + 1,) * 3) if alpha0 is None else np.asarray(alpha0, dtype=np.float64).copy()
    hist = History()

    vals, outs = evaluate_population([pos], q, alpha, spec, obj)
    best = (float(vals[0]), pos.copy(), alpha.copy(), outs[0])
    hist.evaluations += 1
    hist.values.append(best[0])
    hist.stages.append("start")
    hist.thickness.append(outs[0]["t"])
    for rnd in range(rounds):
        # (ii) first-order steps on alpha with the positions held; t follows V*
        a = torch.tensor(alpha, requires_grad=True)
        opt = torch.optim.Adam([a], lr=alpha_lr)
        P = torch.tensor(pos[None], dtype=torch.float64)
        Q = torch.tensor(q[None], dtype=torch.float64)
        for _ in range(alpha_steps):
            opt.zero_grad()
            C, V = AG.Homogenize.apply(P, Q, spec, a)
            L = obj(C, V).sum()
            L.backward()
            hist.evaluations += 1
            val = float(L.detach())
            if val < best[0]:
                best = (val, pos.copy(), a.detach().numpy().copy(), spec.state["last"][0])
            with torch.no_grad():
                a.grad[0, 0, 0] = 0.0  # B_000 = 0: alpha_000 has no effect
            opt.step()
        alpha = a.detach().numpy().copy()
        vals, outs = evaluate_population([pos], q, alpha, spec, obj)
        hist.evaluations += 1
        if vals[0] < best[0]:
            best = (float(vals[0]), pos.copy(), alpha.copy(), outs[0])
        else:
            alpha = best[2].copy()
        hist.values.append(best[0])
        hist.stages.append(f"round {rnd}: alpha")
        hist.thickness.append(best[3]["t"])
        # (iii) CMA-ES on the positions with alpha held
        es = CMAES(pos.ravel(), sigma0, popsize=popsize, seed=seed + rnd)
        for _ in range(cma_generations):
            X = es.ask()
            vals, outs = evaluate_population([x.reshape(-1, 3) for x in X], q, alpha, spec, obj)
            hist.evaluations += len(X)
            k = es.tell(X, vals)
            if vals[k] < best[0]:
                best = (float(vals[k]), np.mod(X[k].reshape(-1, 3), 1.0), alpha.copy(), outs[k])
        pos = best[1].copy()
        hist.values.append(best[0])
        hist.stages.append(f"round {rnd}: positions")
        hist.thickness.append(best[3]["t"])
        if callback:
            callback(rnd, best)
    val, pos, alpha, out = best
    return InverseResult(pos=pos, q=q, alpha=alpha, t=out["t"], value=val, C=out["C"], V=out["V"], history=hist)
