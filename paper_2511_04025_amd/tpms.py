"""Fitting the charge field to a given surface (Sec. 5.3, Eq. (10)).

Targets are implicit periodic surfaces phi(x) = 0 of the unit cell, e.g. the
trigonometric approximations of triply periodic minimal surfaces.  The fit
minimizes, over the charge positions p_m and the spectral weights alpha_hkl,

    L = sum_i F(pbar_i)^2 - lambda sum_i tanh(s F(qbar_i)^2),

where pbar_i are points sampled on the target surface (F should vanish
there), qbar_i points at least a distance d away from it (F should not), and
s is the inverse of the largest |F| over the samples at the current iterate
(a normalization, held constant within a step).  F and dL/d(p_m, q, alpha)
come from the library's point-field entry points; the optimizer (Adam) and the
sampling run on the host.
"""
from dataclasses import dataclass
from typing import Callable

import numpy as np
import torch

TWO_PI = 2.0 * np.pi


# ---- target surfaces: phi and grad phi on (M, 3) points (cell units) ------------
def schwarz_p(x):
    X = TWO_PI * x
    phi = np.cos(X[:, 0]) + np.cos(X[:, 1]) + np.cos(X[:, 2])
    g = -TWO_PI * np.sin(X)
    return phi, g


def gyroid(x):
    X = TWO_PI * x
    s, c = np.sin(X), np.cos(X)
    phi = s[:, 0] * c[:, 1] + s[:, 1] * c[:, 2] + s[:, 2] * c[:, 0]
    g = TWO_PI * np.stack([c[:, 0] * c[:, 1] - s[:, 2] * s[:, 0],
                           -s[:, 0] * s[:, 1] + c[:, 1] * c[:, 2],
                           -s[:, 1] * s[:, 2] + c[:, 2] * c[:, 0]], axis=1)
    return phi, g


def schwarz_d(x):
    X = TWO_PI * x
    s, c = np.sin(X), np.cos(X)
    phi = (s[:, 0] * s[:, 1] * s[:, 2] + s[:, 0] * c[:, 1] * c[:, 2] + c[:, 0] * s[:, 1] * c[:, 2]
           + c[:, 0] * c[:, 1] * s[:, 2])
    gx = c[:, 0] * s[:, 1] * s[:, 2] + c[:, 0] * c[:, 1] * c[:, 2] - s[:, 0] * s[:, 1] * c[:, 2] - s[:, 0] * c[:, 1] * s[:, 2]
    gy = s[:, 0] * c[:, 1] * s[:, 2] - s[:, 0] * s[:, 1] * c[:, 2] + c[:, 0] * c[:, 1] * c[:, 2] - c[:, 0] * s[:, 1] * s[:, 2]
    gz = s[:, 0] * s[:, 1] * c[:, 2] - s[:, 0] * c[:, 1] * s[:, 2] - c[:, 0] * s[:, 1] * s[:, 2] + c[:, 0] * c[:, 1] * c[:, 2]
    return phi, TWO_PI * np.stack([gx, gy, gz], axis=1)


TARGETS = {"P": schwarz_p, "G": gyroid, "D": schwarz_d}


def sample_surface(target: Callable, count, seed=0, newton=30, tol=1e-12):
    """Points on phi = 0: uniform random points moved by Newton steps along
    grad phi (x <- x - phi grad phi / |grad phi|^2) until |phi| <= tol."""
    rng = np.random.default_rng(seed)
    out = []
    while sum(len(o) for o in out) < count:
        x = rng.random((2 * count, 3))
        for _ in range(newton):
            phi, g = target(x)
            gg = np.maximum(np.sum(g * g, axis=1), 1e-30)
            x = x - (phi / gg)[:, None] * g
        phi, g = target(x)
        ok = (np.abs(phi) <= tol) & (np.sum(g * g, axis=1) > 1e-6)
        out.append(np.mod(x[ok], 1.0))
    return np.concatenate(out)[:count]


def sample_off_surface(target: Callable, count, dist=0.05, seed=1):
    """Points whose first-order distance |phi| / |grad phi| to the surface is at
    least `dist` (cell units)."""
    rng = np.random.default_rng(seed)
    out = []
    while sum(len(o) for o in out) < count:
        x = rng.random((4 * count, 3))
        phi, g = target(x)
        d = np.abs(phi) / np.maximum(np.linalg.norm(g, axis=1), 1e-30)
        out.append(x[d >= dist])
    return np.concatenate(out)[:count]


# ---- the field at points as a differentiable function --------------------------
class FieldAtPoints(torch.autograd.Function):
    """F (Eq. (6)) at fixed points as a function of (pos (N, 3), q (N,), alpha
    ((K+1,)*3)); every evaluation and gradient runs in the library."""

    @staticmethod
    def forward(ctx, pos, q, alpha, pts, template):
        from . import api
        d = template.with_(pos=pos.detach().cpu().numpy(), q=q.detach().cpu().numpy(),
                           alpha=alpha.detach().cpu().numpy())
        ctx.design = d
        ctx.pts = pts
        return api.field_points(d, pts).cpu()

    @staticmethod
    def backward(ctx, gF):
        from . import api
        dpos, dq, dal = api.field_points_grad(ctx.design, ctx.pts, gF.detach().to(torch.float64))
        t = lambda a: torch.tensor(a, dtype=torch.float64)
        return t(dpos), t(dq), t(dal), None, None


def fit_loss(F_on, F_off, lam):
    """Eq. (10) with s = 1 / max |F| over both sample sets (held constant)."""
    s = 1.0 / torch.cat([F_on, F_off]).abs().max().detach()
    return (F_on ** 2).sum() - lam * torch.tanh(s * F_off ** 2).sum()


@dataclass
class FitResult:
    pos: np.ndarray
    q: np.ndarray
    alpha: np.ndarray
    loss: list
    surface_residual: float   # mean |F| / max |F| over the surface samples
    separation: float         # share of off-surface samples with |F| > 0.1 max |F|
    target_separation: float  # the same share for the target function itself
    side_agreement: float     # share of off-surface samples on which F and phi (or -phi) agree in sign


def fit_surface(template, target="P", n_on=2048, n_off=2048, dist=0.05, lam=1.0, steps=200, lr=0.01,
                fit_alpha=True, seed=0):
    """Fit the charges (and alpha) of `template` (a workloads.Design: its q
    stay fixed, its positions and alpha move) to a target surface."""
    tf = TARGETS[target] if isinstance(target, str) else target
    on = torch.tensor(sample_surface(tf, n_on, seed=seed))
    off = torch.tensor(sample_off_surface(tf, n_off, dist=dist, seed=seed + 1))
    pts = torch.cat([on, off])
    K1 = template.K + 1
    pos = torch.tensor(np.asarray(template.pos, dtype=np.float64), requires_grad=True)
    q = torch.tensor(np.asarray(template.q, dtype=np.float64))
    al0 = np.ones((K1,) * 3) if template.alpha is None else np.asarray(template.alpha, dtype=np.float64)
    alpha = torch.tensor(al0, requires_grad=fit_alpha)
    opt = torch.optim.Adam([pos, alpha] if fit_alpha else [pos], lr=lr)
    hist = []
    for _ in range(steps):
        opt.zero_grad()
        F = FieldAtPoints.apply(pos, q, alpha, pts, template)
        L = fit_loss(F[:n_on], F[n_on:], lam)
        L.backward()
        hist.append(float(L.detach()))
        opt.step()
    with torch.no_grad():
        F = FieldAtPoints.apply(pos, q, alpha, pts, template)
        m = float(F.abs().max())
        res = float(F[:n_on].abs().mean()) / m
        sep = float((F[n_on:].abs() > 0.1 * m).double().mean())
        sF = np.sign(F[n_on:].numpy())
    phi = tf(off.numpy())[0]
    tsep = float(np.mean(np.abs(phi) > 0.1 * np.abs(phi).max()))
    agree = float(np.mean(sF == np.sign(phi)))
    return FitResult(pos=np.mod(pos.detach().numpy(), 1.0), q=q.numpy(), alpha=alpha.detach().numpy(), loss=hist,
                     surface_residual=res, separation=sep, target_separation=tsep,
                     side_agreement=max(agree, 1.0 - agree))
