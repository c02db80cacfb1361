"""Pins of the oracle's sensitivities (Eq. (9)) against finite differences,
the Euler identity of a 1-homogeneous function and charge-scale invariance."""
import numpy as np
import pytest

from oracle import adjoint as adj, fem, homogenize as hom, metrics
from paper_2511_04025_amd import workloads as wl

NU = 0.3


def test_energy_sensitivity_matches_finite_differences_and_euler_rule():
    n = 4
    rng = np.random.default_rng(1)
    Ee = np.where(rng.random((n, n, n)) < 0.5, 1.0, 0.05)
    C, info = hom.homogenize_stiffness(Ee, NU, solver="direct")
    J = adj.element_energy_jacobian(info["U"], NU, n)  # (n^3, 6, 6)
    # Euler: C is 1-homogeneous in the moduli, so sum_e E_e dC/dE_e = C
    assert np.max(np.abs(np.einsum("e,eij->ij", Ee.ravel(), J) - C)) < 1e-13
    h = 1e-6
    for e in (0, 17, 42):
        Ep = Ee.copy().ravel()
        Em = Ee.copy().ravel()
        Ep[e] += h
        Em[e] -= h
        Cp, _ = hom.homogenize_stiffness(Ep.reshape(n, n, n), NU, solver="direct")
        Cm, _ = hom.homogenize_stiffness(Em.reshape(n, n, n), NU, solver="direct")
        fd = (Cp - Cm) / (2 * h)
        assert np.max(np.abs(fd - J[e])) < 1e-6 * np.abs(J[e]).max()


def test_loss_gradient_wrt_C_matches_finite_differences():
    d = wl.random_design(41, 6, N=8, vf=0.3, E_void=1e-2)
    C, _ = hom.homogenize_design(d.pos, d.q, 6, target_vf=0.3, E_void=1e-2, solver="direct")
    Kt, nut = 0.05, 0.1
    g = adj.bulk_poisson_loss_grad(C, Kt, nut)
    h = 1e-7
    for i in range(6):
        for j in range(6):
            Cp = C.copy()
            Cm = C.copy()
            Cp[i, j] += h
            Cm[i, j] -= h
            fd = (metrics.bulk_poisson_loss(Cp, Kt, nut) - metrics.bulk_poisson_loss(Cm, Kt, nut)) / (2 * h)
            assert abs(fd - g[i, j]) < 1e-6 * np.abs(g).max() + 1e-9, (i, j)


def _loss(pos, q, n, t, kappa, E_void, dLdC, dLdV):
    C, info = hom.homogenize_design(pos, q, n, thickness=t, kappa=kappa, E_void=E_void, solver="direct")
    return np.sum(dLdC * C) + dLdV * info["V"], C, info


def test_design_gradient_matches_central_differences():
    # a linear functional L = <G, C> + g V of the outputs exercises every path
    n = 8
    d = wl.random_design(43, n, N=6, vf=0.2, E_void=1e-3)
    kappa = 4.0 * n
    from oracle import field as fld
    F, G = fld.field_and_gradient(d.pos, d.q, n)
    t = fld.thickness_for_volume(fld.distance(F, G), 0.25, kappa)
    rng = np.random.default_rng(5)
    dLdC = rng.standard_normal((6, 6))
    dLdC = dLdC + dLdC.T
    dLdV = 0.7
    L0, C0, info = _loss(d.pos, d.q, n, t, kappa, d.E_void, dLdC, dLdV)
    dpos, dq = adj.design_gradient(info, d.pos, d.q, n, dLdC, dLdV, kappa=kappa, E_void=d.E_void)
    # small step: d = |F| / ||grad F|| has a kink where F crosses zero at a
    # voxel center; h = 1e-6 keeps every voxel on one side of it, and the
    # direct solver keeps the differences exact to ~1e-10
    h = 1e-6
    checks = [("pos", 0, 0), ("pos", 2, 1), ("pos", 4, 2), ("q", 1, None), ("q", 5, None)]
    for kind, j, ax in checks:
        pp, pm = d.pos.copy(), d.pos.copy()
        qp, qm = d.q.copy(), d.q.copy()
        if kind == "pos":
            pp[j, ax] += h
            pm[j, ax] -= h
            ref = dpos[j, ax]
        else:
            qp[j] += h
            qm[j] -= h
            ref = dq[j]
        Lp = _loss(pp, qp, n, t, kappa, d.E_void, dLdC, dLdV)[0]
        Lm = _loss(pm, qm, n, t, kappa, d.E_void, dLdC, dLdV)[0]
        fd = (Lp - Lm) / (2 * h)
        scale = max(np.abs(dpos).max(), np.abs(dq).max())
        assert abs(fd - ref) < 1e-7 * scale, (kind, j, ax, fd, ref)
    # F scales with q, d does not (iso = 0), so the loss is flat along q
    assert abs(np.dot(d.q, dq)) < 1e-10 * np.abs(dq).max() * np.abs(d.q).sum()


def test_hard_step_rejected():
    with pytest.raises(ValueError):
        adj.voxel_sensitivities(np.zeros((2, 2, 2)), np.zeros((3, 2, 2, 2)), np.zeros((2, 2, 2)),
                                np.zeros((2, 2, 2)), 0.1, 0.0, 1.0, 0.0, np.zeros((2, 2, 2)), 0.0)


def _loss_full(pos, q, n, t, kappa, E_void, dLdC, dLdV, alpha):
    C, info = hom.homogenize_design(pos, q, n, thickness=t, kappa=kappa, E_void=E_void, alpha=alpha,
                                    solver="direct")
    return np.sum(dLdC * C) + dLdV * info["V"], info


def _setup_full(n=8, seed=47):
    from oracle import field as fld
    d = wl.random_design(seed, n, N=6, vf=0.2, E_void=1e-3)
    kappa = 4.0 * n
    alpha = 1.0 + 0.3 * np.random.default_rng(seed).standard_normal((4, 4, 4))
    F, G = fld.field_and_gradient(d.pos, d.q, n, alpha=alpha)
    t = fld.thickness_for_volume(fld.distance(F, G), 0.25, kappa)
    rng = np.random.default_rng(6)
    dLdC = rng.standard_normal((6, 6))
    dLdC = dLdC + dLdC.T
    return d, kappa, alpha, t, dLdC, 0.7


def test_alpha_and_thickness_gradients_match_central_differences():
    # Eq. (9) for theta = alpha_hkl and theta = t, against central differences
    # of a linear functional of (C^H, V) (direct solves, h = 1e-6)
    n = 8
    d, kappa, alpha, t, dLdC, dLdV = _setup_full(n)
    _, info = _loss_full(d.pos, d.q, n, t, kappa, d.E_void, dLdC, dLdV, alpha)
    dpos, dq, dalpha, dt = adj.design_gradient_full(info, d.pos, d.q, n, dLdC, dLdV, alpha=alpha,
                                                    kappa=kappa, E_void=d.E_void)
    h = 1e-6
    scale = np.abs(dalpha).max()
    for (a, b, c) in ((0, 0, 1), (1, 2, 3), (3, 0, 0), (2, 2, 0)):
        ap, am = alpha.copy(), alpha.copy()
        ap[a, b, c] += h
        am[a, b, c] -= h
        fd = (_loss_full(d.pos, d.q, n, t, kappa, d.E_void, dLdC, dLdV, ap)[0] -
              _loss_full(d.pos, d.q, n, t, kappa, d.E_void, dLdC, dLdV, am)[0]) / (2 * h)
        assert abs(fd - dalpha[a, b, c]) < 1e-7 * scale, ((a, b, c), fd, dalpha[a, b, c])
    assert dalpha[0, 0, 0] == 0.0
    fd = (_loss_full(d.pos, d.q, n, t + h, kappa, d.E_void, dLdC, dLdV, alpha)[0] -
          _loss_full(d.pos, d.q, n, t - h, kappa, d.E_void, dLdC, dLdV, alpha)[0]) / (2 * h)
    assert abs(fd - dt) < 1e-7 * abs(dt), (fd, dt)
    # F is linear in alpha and d = |F| / ||grad F|| is invariant to scaling F,
    # so the loss is flat along alpha itself
    assert abs(np.sum(alpha * dalpha)) < 1e-10 * np.abs(alpha * dalpha).sum()
    # the same position and charge gradients as the fixed-thickness routine
    dpos0, dq0 = adj.design_gradient(info, d.pos, d.q, n, dLdC, dLdV, alpha=alpha, kappa=kappa,
                                     E_void=d.E_void)
    assert np.array_equal(dpos0, dpos) and np.array_equal(dq0, dq)


def test_volume_constrained_gradient_matches_differences_with_bisection():
    # t re-solved by bisection for the target volume at every perturbed design
    # (Sec. 4.3's joint optimization): the implicit-function gradient against
    # central differences of the constrained loss
    from oracle import field as fld
    n = 8
    d, kappa, alpha, _, dLdC, _ = _setup_full(n, seed=53)
    V_star = 0.25

    def constrained_loss(pos, al):
        F, G = fld.field_and_gradient(pos, d.q, n, alpha=al)
        t = fld.thickness_for_volume(fld.distance(F, G), V_star, kappa)
        return _loss_full(pos, d.q, n, t, kappa, d.E_void, dLdC, 0.0, al)

    L0, info = constrained_loss(d.pos, alpha)
    assert abs(info["V"] - V_star) <= 1e-12
    gL = adj.design_gradient_full(info, d.pos, d.q, n, dLdC, 0.0, alpha=alpha, kappa=kappa, E_void=d.E_void)
    gV = adj.design_gradient_full(info, d.pos, d.q, n, np.zeros((6, 6)), 1.0, alpha=alpha, kappa=kappa,
                                  E_void=d.E_void)
    dpos, dq, dalpha = adj.volume_constrained(gL, gV)
    h = 1e-5
    scale = max(np.abs(dpos).max(), np.abs(dalpha).max())
    for kind, idx in (("pos", (1, 0)), ("pos", (3, 2)), ("alpha", (1, 1, 0)), ("alpha", (0, 2, 3))):
        pp, pm = d.pos.copy(), d.pos.copy()
        ap, am = alpha.copy(), alpha.copy()
        if kind == "pos":
            pp[idx] += h
            pm[idx] -= h
            ref = dpos[idx]
        else:
            ap[idx] += h
            am[idx] -= h
            ref = dalpha[idx]
        fd = (constrained_loss(pp, ap)[0] - constrained_loss(pm, am)[0]) / (2 * h)
        assert abs(fd - ref) < 2e-6 * scale, (kind, idx, fd, ref)
