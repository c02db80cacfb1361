"""Pins of the oracle's multigrid coarse grids against closed forms."""
import numpy as np

from oracle import fem, multigrid as mg


def test_prolongation_interpolates():
    nc = 4
    P = mg.prolongation(nc)
    nf = 2 * nc
    assert P.shape == (3 * nf ** 3, 3 * nc ** 3)
    # constants are reproduced, per component
    for c in range(3):
        u = np.zeros(3 * nc ** 3)
        u[c::3] = 1.0
        v = P @ u
        assert np.allclose(v[c::3], 1.0) and np.allclose(np.delete(v, np.s_[c::3]), 0.0)
    # a coarse field linear in x on the nodes 0..nc-1 is interpolated linearly
    # between them (away from the periodic seam)
    X = np.arange(nc, dtype=float)
    u = np.zeros((nc, nc, nc, 3))
    u[..., 1] = 2.0 * X[None, None, :] + 0.5
    v = (P @ u.ravel()).reshape(nf, nf, nf, 3)
    xf = np.arange(nf - 1) / 2.0
    assert np.allclose(v[3, 2, : nf - 1, 1], 2.0 * xf + 0.5)
    # rows sum to 1 per component, columns to 8 (each coarse node spreads over 27 fine nodes)
    Pc = P[0::3, 0::3]
    assert np.allclose(np.asarray(Pc.sum(axis=1)).ravel(), 1.0)
    assert np.allclose(np.asarray(Pc.sum(axis=0)).ravel(), 8.0)


def test_galerkin_of_uniform_moduli_is_the_coarse_stiffness():
    # on a uniform material the coarse Q1 space is a subspace of the fine one,
    # so P^T K_h P is the stiffness of the coarse mesh, whose element of edge 2
    # has matrix 2 K_0 in unit-element coordinates
    n, nu, E = 6, 0.27, 1.7
    K = fem.assemble(np.full(n ** 3, E), nu, n)
    Kc = mg.galerkin(K, n)
    ref = fem.assemble(np.full((n // 2) ** 3, 2.0 * E), nu, n // 2)
    assert abs(Kc - ref).max() <= 1e-12 * abs(ref).max()


def test_galerkin_keeps_symmetry_and_rigid_modes():
    n = 8
    rng = np.random.default_rng(4)
    E = np.where(rng.random(n ** 3) < 0.3, 1.0, 1e-3)
    Kc = mg.galerkin(fem.assemble(E, 0.3, n), n)
    assert abs(Kc - Kc.T).max() <= 1e-14 * abs(Kc).max()
    for c in range(3):
        t = np.zeros(Kc.shape[0])
        t[c::3] = 1.0
        assert np.abs(Kc @ t).max() <= 1e-13 * abs(Kc).max()
    # positive semidefinite: x^T Kc x = (P x)^T K (P x) >= 0
    x = rng.standard_normal(Kc.shape[0])
    assert x @ (Kc @ x) > 0
