"""Pins of the oracle's element matrix, assembly, load vectors and solvers."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import fem, solve as slv


NU = 0.3


def test_element_stiffness_invariants():
    K0 = fem.element_stiffness(NU)
    lam, mu = fem.lame(1.0, NU)
    assert np.max(np.abs(K0 - K0.T)) < 1e-15
    # every diagonal entry is (lambda + 4 mu) / 9 (for E = 1, nu = 0.3: 0.2350427...)
    assert np.max(np.abs(np.diag(K0) - (lam + 4 * mu) / 9.0)) < 1e-15
    assert abs((lam + 4 * mu) / 9.0 - 0.23504273504273504) < 1e-15
    ev = np.linalg.eigvalsh(K0)
    assert np.sum(ev < 1e-12) == 6 and np.min(ev) > -1e-14  # rank 18, PSD
    # the 6 rigid modes: 3 translations and 3 infinitesimal rotations
    X = fem.CORNERS.astype(float)
    for c in range(3):
        t = np.zeros(24)
        t[c::3] = 1.0
        assert np.max(np.abs(K0 @ t)) < 1e-14
    for w in np.eye(3):
        rot = np.cross(w[None, :], X).ravel()
        assert np.max(np.abs(K0 @ rot)) < 1e-14


def test_uniform_strain_energy_is_D():
    # a linear field chi^k = eps^k x is reproduced exactly by the trilinear
    # element, so its element energy is the material matrix: chi^i K_0 chi^j = D_ij
    K0 = fem.element_stiffness(NU)
    chi = fem.test_displacements()
    assert np.max(np.abs(chi.T @ K0 @ chi - fem.isotropic_D(1.0, NU))) < 1e-14


def test_isotropic_D_values():
    D = fem.isotropic_D(1.0, 0.3)
    assert abs(D[0, 0] - 1.3461538461538463) < 1e-15
    assert abs(D[0, 1] - 0.5769230769230769) < 1e-15
    assert abs(D[3, 3] - 0.38461538461538464) < 1e-15
    # inverse: uniaxial compliance 1/E and Poisson ratio
    S = np.linalg.inv(D)
    assert abs(1.0 / S[0, 0] - 1.0) < 1e-14 and abs(-S[0, 1] / S[0, 0] - 0.3) < 1e-14


@pytest.mark.parametrize("n", [2, 3, 5])
def test_assembly_structure(n):
    rng = np.random.default_rng(n)
    Ee = rng.uniform(0.1, 2.0, (n, n, n))
    K = fem.assemble(Ee, NU, n)
    assert abs(K - K.T).max() < 1e-14
    for c in range(3):
        t = np.zeros(3 * n ** 3)
        t[c::3] = 1.0
        assert np.max(np.abs(K @ t)) < 1e-13
    if n >= 3:
        assert np.max(np.diff(K.indptr)) == 81
    # diagonal: (lambda + 4 mu)/9 times the sum of the 8 incident element moduli
    lam, mu = fem.lame(1.0, NU)
    s = np.zeros((n, n, n))
    for az in (0, 1):
        for ay in (0, 1):
            for ax in (0, 1):
                s += np.roll(Ee, (az, ay, ax), axis=(0, 1, 2))
    assert np.max(np.abs(K.diagonal()[0::3] - (lam + 4 * mu) / 9.0 * s.ravel())) < 1e-13
    f = fem.load_vectors(Ee, NU, n)
    for c in range(3):
        assert np.max(np.abs(f[c::3].sum(axis=0))) < 1e-13
    # homogeneous material: a uniform strain is already in equilibrium
    f0 = fem.load_vectors(np.full((n, n, n), 1.7), NU, n)
    assert np.max(np.abs(f0)) < 1e-14


def test_brute_force_assembly_tiny():
    # n = 2: write K entry by entry with explicit loops over elements and corners
    n = 2
    rng = np.random.default_rng(4)
    Ee = rng.uniform(0.5, 1.5, (n, n, n))
    K0 = fem.element_stiffness(NU)
    ref = np.zeros((3 * n ** 3, 3 * n ** 3))
    for k in range(n):
        for j in range(n):
            for i in range(n):
                nodes = []
                for a in range(8):
                    ax, ay, az = a & 1, (a >> 1) & 1, (a >> 2) & 1
                    nodes.append((((k + az) % n) * n + (j + ay) % n) * n + (i + ax) % n)
                for a in range(8):
                    for b in range(8):
                        for c in range(3):
                            for d in range(3):
                                ref[3 * nodes[a] + c, 3 * nodes[b] + d] += Ee[k, j, i] * K0[3 * a + c, 3 * b + d]
    K = fem.assemble(Ee, NU, n).toarray()
    assert np.max(np.abs(K - ref)) < 1e-14


def test_cg_matches_direct_solve():
    n = 6
    rng = np.random.default_rng(9)
    Ee = np.where(rng.random((n, n, n)) < 0.4, 1.0, 1e-3)
    K = fem.assemble(Ee, NU, n)
    f = fem.load_vectors(Ee, NU, n)
    Kp, fp = slv.pin_node0(K, f)
    u_cg, iters, res = slv.pcg_jacobi(Kp, fp, rtol=1e-12)
    u_lu = slv.direct_solve(Kp, fp)
    assert np.all(res < 2e-12)
    assert np.all(iters > 0)
    assert np.max(np.abs(u_cg - u_lu)) < 1e-8 * np.max(np.abs(u_lu))
    assert np.all(u_lu[:3] == 0.0)
    # the pinned and the singular systems agree up to a rigid translation
    r = f - K @ u_lu
    assert np.max(np.abs(r)) < 1e-10


def test_cg_zero_rhs():
    n = 3
    K = fem.assemble(np.ones((n, n, n)), NU, n)
    Kp, fp = slv.pin_node0(K, np.zeros((3 * n ** 3, 6)))
    u, iters, res = slv.pcg_jacobi(Kp, fp)
    assert np.all(u == 0.0) and np.all(iters == 0)


def test_stiffness_rows_match_assembly_and_rigid_modes():
    # rows of K u by the per-node definition equal the assembled product
    n, nu = 5, 0.27
    rng = np.random.default_rng(31)
    E = rng.uniform(1e-3, 1.0, n ** 3)
    U = rng.standard_normal((3 * n ** 3, 2))
    Q = fem.assemble(E, nu, n) @ U
    nodes = np.array([0, 1, n - 1, n * n - 1, n ** 3 - 1, 37, 64, 99])
    u_at = lambda ids: U.reshape(n ** 3, 3, 2)[ids]
    rows = fem.stiffness_rows(E, nu, n, u_at, nodes)
    assert np.max(np.abs(rows - Q.reshape(n ** 3, 3, 2)[nodes])) <= 1e-13 * np.abs(Q).max()
    # a rigid translation has no force anywhere
    t = np.tile(np.array([0.3, -1.2, 2.0])[None, :, None], (n ** 3, 1, 1))
    rows = fem.stiffness_rows(E, nu, n, lambda ids: t[ids], np.arange(n ** 3))
    assert np.abs(rows).max() <= 1e-14 * np.abs(E).max()
    # a single displaced node pulls on itself with the diagonal closed form:
    # (lambda + 4 mu) / 9 times the sum of its 8 incident E_e (E = 1 units)
    lam, mu = fem.lame(1.0, nu)
    k = 62
    vx, vy, vz = k % n, (k // n) % n, k // (n * n)
    s = sum(E[(((vz - az) % n) * n + (vy - ay) % n) * n + (vx - ax) % n] for ax, ay, az in fem.CORNERS)
    e = np.zeros((n ** 3, 3, 1))
    e[k, 1, 0] = 1.0
    rows = fem.stiffness_rows(E, nu, n, lambda ids: e[ids], np.array([k]))
    assert abs(rows[0, 1, 0] - (lam + 4 * mu) / 9 * s) <= 1e-14
