"""Design sensitivities of C^H and V (oracle, FP64).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Eq. (9): dL/dtheta = sum_e (dL/dC^H : dC^H/dbeta_e) dbeta_e/dtheta.
Because every u^(k) is at equilibrium, the energy form is stationary in u and
    dC_ij / dE_e = (1/n^3) (chi^i + u^i_e)^T K_0 (chi^j + u^j_e)
(no adjoint solve).  dbeta_e/dtheta follows from the logistic occupancy of
Sec. 4.1, the distance d = |F - c| / ||grad F|| of Eq. (7) and the charge field
of Eq. (6); the parameters are the charge positions and values, the
spectral weights alpha_hkl and the half-thickness t (Sec. 4.3 lists all
three), the last either free or tied to a target volume by the implicit
function theorem.  The hard step has no useful derivative and is rejected.

Conventions at kinks: sgn(0) = 0 where F = c; where the gradient norm is
clamped at its floor the clamped value is treated as a constant.
"""
import numpy as np

from . import fem
from . import field as fld
from .homogenize import element_vectors


def element_energy_weights(Ee, U, nu, n, dL_dC):
    """s_e = sum_ij dL/dC_ij * dC_ij/dE_e for every element, shape (n,n,n)."""
    K0 = fem.element_stiffness(nu)
    V = element_vectors(U, n)
    W = np.einsum("ab,ebj->eaj", K0, V)
    s = np.einsum("ij,eai,eaj->e", np.asarray(dL_dC, dtype=np.float64), V, W) / n ** 3
    return s.reshape(n, n, n)


def element_energy_jacobian(U, nu, n):
    """dC_ij/dE_e for every element: shape (n^3, 6, 6) (small grids only)."""
    K0 = fem.element_stiffness(nu)
    V = element_vectors(U, n)
    W = np.einsum("ab,ebj->eaj", K0, V)
    return np.einsum("eai,eaj->eij", V, W) / n ** 3


def voxel_sensitivities(F, G, d, beta, t, kappa, E, E_void, s_e, dL_dV, iso=0.0, dist_mode=0):
    """Per-voxel adjoint fields (g_F, g_G): dL/dF_e and dL/d(grad F)_e.

    dL/dbeta_e = s_e (E - E_void) + dL/dV / n^3;  dbeta/dd = -kappa beta (1 - beta);
    dd/dF = sgn(F - c) / ||grad F||;  dd/dgrad F = -|F - c| grad F / ||grad F||^3.
    """
    if kappa <= 0:
        raise ValueError("the hard step has no gradient; use kappa > 0")
    n = F.shape[0]
    gbeta = s_e * (E - E_void) + dL_dV / n ** 3
    gd = gbeta * (-kappa * beta * (1.0 - beta))
    sgn = np.sign(F - iso)
    if dist_mode == 1:
        return gd * sgn, np.zeros_like(G)
    gn = np.sqrt(G[0] ** 2 + G[1] ** 2 + G[2] ** 2)
    gmin = 1e-12 * gn.max()
    clamped = gn < gmin
    den = np.maximum(gn, gmin)
    gF = gd * sgn / den
    num = np.abs(F - iso)
    gG = np.where(clamped[None], 0.0, -(gd * num / den ** 3)[None] * G)
    return gF, gG


def charge_gradients(gF, gG, pos, q, n, K=3, alpha=None):
    """Pull (g_F, g_G) back onto the charges by direct summation over every
    (charge, mode) term of Eq. (6).  Returns (dL/dpos (N,3), dL/dq (N,))."""
    pos = np.asarray(pos, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    a = np.ones((K + 1,) * 3) if alpha is None else np.asarray(alpha, dtype=np.float64).reshape((K + 1,) * 3)
    c = fld.voxel_centers(n)
    tp = 2.0 * np.pi
    dpos = np.zeros_like(pos)
    dq = np.zeros_like(q)

    def outer(fz, fy, fx):
        return fz[:, None, None] * fy[None, :, None] * fx[None, None, :]

    for j in range(len(q)):
        for (h, k, l) in fld.modes(K):
            coef = a[h, k, l] * fld.mode_weight(h, k, l) / (h * h + k * k + l * l)
            if coef == 0.0:
                continue
            ax, ay, az = tp * h * (c - pos[j, 0]), tp * k * (c - pos[j, 1]), tp * l * (c - pos[j, 2])
            cx, cy, cz = np.cos(ax), np.cos(ay), np.cos(az)
            dx, dy, dz = -tp * h * np.sin(ax), -tp * k * np.sin(ay), -tp * l * np.sin(az)
            ddx, ddy, ddz = -(tp * h) ** 2 * cx, -(tp * k) ** 2 * cy, -(tp * l) ** 2 * cz
            phi = coef * outer(cz, cy, cx)
            px, py, pz = coef * outer(cz, cy, dx), coef * outer(cz, dy, cx), coef * outer(dz, cy, cx)
            pxx, pyy, pzz = coef * outer(cz, cy, ddx), coef * outer(cz, ddy, cx), coef * outer(ddz, cy, cx)
            pxy, pxz, pyz = coef * outer(cz, dy, dx), coef * outer(dz, cy, dx), coef * outer(dz, dy, cx)
            dq[j] += np.sum(gF * phi + gG[0] * px + gG[1] * py + gG[2] * pz)
            # F depends on x - x_j, so d/dx_j = -d/dx
            dpos[j, 0] -= q[j] * np.sum(gF * px + gG[0] * pxx + gG[1] * pxy + gG[2] * pxz)
            dpos[j, 1] -= q[j] * np.sum(gF * py + gG[0] * pxy + gG[1] * pyy + gG[2] * pyz)
            dpos[j, 2] -= q[j] * np.sum(gF * pz + gG[0] * pxz + gG[1] * pyz + gG[2] * pzz)
    return dpos, dq


def alpha_gradients(gF, gG, pos, q, n, K=3):
    """Pull (g_F, g_G) back onto the spectral weights: Eq. (6) is linear in
    alpha, so dF/dalpha_hkl = w_hkl / (h^2+k^2+l^2) sum_j q_j cos cos cos and
    d(grad F)/dalpha_hkl is its gradient.  Direct summation over every (charge,
    mode) term; returns dL/dalpha of shape (K+1, K+1, K+1), entry (0,0,0) zero
    (B_000 = 0)."""
    pos = np.asarray(pos, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    c = fld.voxel_centers(n)
    tp = 2.0 * np.pi
    out = np.zeros((K + 1,) * 3)

    def outer(fz, fy, fx):
        return fz[:, None, None] * fy[None, :, None] * fx[None, None, :]

    for (h, k, l) in fld.modes(K):
        base = fld.mode_weight(h, k, l) / (h * h + k * k + l * l)
        acc = 0.0
        for j in range(len(q)):
            ax, ay, az = tp * h * (c - pos[j, 0]), tp * k * (c - pos[j, 1]), tp * l * (c - pos[j, 2])
            cx, cy, cz = np.cos(ax), np.cos(ay), np.cos(az)
            dx, dy, dz = -tp * h * np.sin(ax), -tp * k * np.sin(ay), -tp * l * np.sin(az)
            acc += q[j] * np.sum(gF * outer(cz, cy, cx) + gG[0] * outer(cz, cy, dx) +
                                 gG[1] * outer(cz, dy, cx) + gG[2] * outer(dz, cy, cx))
        out[h, k, l] = base * acc
    return out


def thickness_gradient(s_e, beta, kappa, E, E_void, dL_dV):
    """dL/dt with t a free parameter: beta = 1 / (1 + exp(-kappa (t - d))) gives
    dbeta/dt = kappa beta (1 - beta), and dL/dbeta_e = s_e (E - E_void) + dL/dV / n^3."""
    if kappa <= 0:
        raise ValueError("the hard step has no gradient; use kappa > 0")
    n = beta.shape[0]
    gbeta = s_e * (E - E_void) + dL_dV / n ** 3
    return float(np.sum(gbeta * kappa * beta * (1.0 - beta)))


def design_gradient_full(info, pos, q, n, dL_dC, dL_dV, *, K=3, alpha=None, iso=0.0,
                         kappa, dist_mode=0, E=1.0, nu=0.3, E_void=1e-3):
    """Eq. (9) for every design parameter theta in {charge positions, charge
    values, alpha_hkl, t} (t held as an independent parameter): returns
    (dL/dpos (N,3), dL/dq (N,), dL/dalpha (K+1,K+1,K+1), dL/dt)."""
    s_e = element_energy_weights(info["Ee"], info["U"], nu, n, dL_dC)
    gF, gG = voxel_sensitivities(info["F"], info["G"], info["d"], info["beta"], info["t"],
                                 kappa, E, E_void, s_e, dL_dV, iso=iso, dist_mode=dist_mode)
    dpos, dq = charge_gradients(gF, gG, pos, q, n, K=K, alpha=alpha)
    dalpha = alpha_gradients(gF, gG, pos, q, n, K=K)
    dt = thickness_gradient(s_e, info["beta"], kappa, E, E_void, dL_dV)
    return dpos, dq, dalpha, dt


def volume_constrained(grad_L, grad_V):
    """Gradient of L along the volume constraint V(theta, t) = V* with t
    re-solved for every theta (Sec. 4.3's joint optimization, where t is set
    by bisection): by the implicit function theorem dt/dtheta = -(dV/dtheta) /
    (dV/dt), so dL/dtheta|_V = dL/dtheta - (dL/dt / dV/dt) dV/dtheta.  grad_L
    and grad_V are (dpos, dq, dalpha, dt) tuples of design_gradient_full for
    (dL/dC, dL/dV) and for (0, 1); returns (dpos, dq, dalpha)."""
    r = grad_L[3] / grad_V[3]
    return tuple(gl - r * gv for gl, gv in zip(grad_L[:3], grad_V[:3]))


def design_gradient(info, pos, q, n, dL_dC, dL_dV, *, K=3, alpha=None, iso=0.0,
                    kappa, dist_mode=0, E=1.0, nu=0.3, E_void=1e-3):
    """dL/dpos, dL/dq for a forward result ``info`` of homogenize_design, given
    the upstream gradients dL/dC (6x6) and dL/dV."""
    s_e = element_energy_weights(info["Ee"], info["U"], nu, n, dL_dC)
    gF, gG = voxel_sensitivities(info["F"], info["G"], info["d"], info["beta"], info["t"],
                                 kappa, E, E_void, s_e, dL_dV, iso=iso, dist_mode=dist_mode)
    return charge_gradients(gF, gG, pos, q, n, K=K, alpha=alpha)


# ---------------------------------------------------------------------------
# gradient of the bulk-modulus / Poisson-ratio objective with respect to C
# ---------------------------------------------------------------------------

_A_BULK = np.zeros((6, 6))
_A_BULK[:3, :3] = 1.0


def _weighted_sum_grad_inv(S, A):
    """d/dC of sum_ij A_ij (C^-1)_ij, using dS = -S dC S."""
    return -S.T @ A @ S.T


def bulk_poisson_loss_grad(C, K_target, nu_target, w_K=1.0, w_nu=1.0):
    """dL/dC (6x6) of metrics.bulk_poisson_loss, written with every sum over the
    full 3x3 normal block so that the result does not assume C symmetric."""
    C = np.asarray(C, dtype=np.float64)
    S = np.linalg.inv(C)
    # Voigt: K_V = sum_{i,j<3} C_ij / 9 ; G_V = (tr_n C - (1/2) offsum_n C + 3 tr_s C) / 15
    KV = (_A_BULK * C).sum() / 9.0
    dKV = _A_BULK / 9.0
    A_GV = np.zeros((6, 6))
    A_GV[:3, :3] = -0.5
    for i in range(3):
        A_GV[i, i] = 1.0
    for i in range(3, 6):
        A_GV[i, i] = 3.0
    GV = (A_GV * C).sum() / 15.0
    dGV = A_GV / 15.0
    # Reuss: K_R = 1 / sum_{i,j<3} S_ij ; G_R = 15 / (4 tr_n S - 2 offsum_n S + 3 tr_s S)
    a = (_A_BULK * S).sum()
    KR = 1.0 / a
    dKR = -(1.0 / a ** 2) * _weighted_sum_grad_inv(S, _A_BULK)
    A_GR = np.zeros((6, 6))
    A_GR[:3, :3] = -2.0
    for i in range(3):
        A_GR[i, i] = 4.0
    for i in range(3, 6):
        A_GR[i, i] = 3.0
    b = (A_GR * S).sum()
    GR = 15.0 / b
    dGR = -(15.0 / b ** 2) * _weighted_sum_grad_inv(S, A_GR)
    KH, GH = 0.5 * (KV + KR), 0.5 * (GV + GR)
    dKH, dGH = 0.5 * (dKV + dKR), 0.5 * (dGV + dGR)
    nu = (3.0 * KH - 2.0 * GH) / (2.0 * (3.0 * KH + GH))
    # dnu/dK and dnu/dG of nu = (3K - 2G) / (2 (3K + G))
    den = 2.0 * (3.0 * KH + GH) ** 2
    dnu_dK = (3.0 * (3.0 * KH + GH) - 3.0 * (3.0 * KH - 2.0 * GH)) / den
    dnu_dG = (-2.0 * (3.0 * KH + GH) - (3.0 * KH - 2.0 * GH)) / den
    dnu = dnu_dK * dKH + dnu_dG * dGH
    return (2.0 * w_K * (KV / K_target - 1.0) / K_target) * dKV + (2.0 * w_nu * (nu - nu_target)) * dnu
