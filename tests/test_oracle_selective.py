"""Pins of the selective (culled) oracle, Sec. 4.2.

Closed forms: a laminate whose void layers are culled leaves free plates,
whose in-plane tensor is the plane-stress one scaled by the solid fraction and
whose out-of-plane entries vanish (the trilinear element holds the exact,
piecewise-linear solution); a fully solid cell returns the base tensor.
Limits: the dense oracle with the stiffness floor E_void -> 0 tends to the
culled result.  Brute force: the active-node rule at n = 4, and a direct
solve with one node pinned per connected piece.  Invariants: octahedral
charge sets give cubic C^H; the Voigt bound.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fem, field as fld, homogenize as hom, selective as sel
from paper_2511_04025_amd import workloads as wl

NU = 0.3


def plate_tensor(fs, E=1.0, nu=NU, axis=2):
    """Free isotropic plates normal to `axis` with solid fraction fs: in-plane
    plane-stress stiffness times fs, zero for every entry that strains or
    shears across the plates."""
    lam, mu = fem.lame(E, nu)
    P = lam + 2 * mu
    C = np.zeros((6, 6))
    inplane = [a for a in range(3) if a != axis]
    for a in inplane:
        C[a, a] = fs * (P - lam * lam / P)
    a, b = inplane
    C[a, b] = C[b, a] = fs * (lam - lam * lam / P)
    shear_in = {frozenset((0, 1)): 5, frozenset((0, 2)): 4, frozenset((1, 2)): 3}[frozenset(inplane)]
    C[shear_in, shear_in] = fs * mu
    return C


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_culled_laminate_gives_free_plates(axis):
    # two separated plates (layers 0-1 and 3); layers 2, 4, 5 culled
    n = 6
    prof = np.array([1.0, 1.0, 0.0, 1.0, 0.0, 0.0])
    shape = [1, 1, 1]
    shape[2 - axis] = n
    beta = np.broadcast_to(prof.reshape(shape), (n, n, n)).copy()
    C, info = sel.homogenize_selective_stiffness(sel.culled_moduli(beta), NU)
    ref = plate_tensor(0.5, axis=axis)
    assert np.max(np.abs(C - ref)) < 1e-11, np.abs(C - ref).max()
    # active nodes: the node planes of the two plates (3 + 2 of 6)
    assert info["n_active_nodes"] == 5 * n * n
    assert info["n_active_voxels"] == 3 * n * n


def test_direct_solve_with_one_pin_per_piece_matches_cg():
    # the plates wrap around the cell in-plane, so each piece has only the
    # three translations: pinning one node per piece makes K nonsingular
    n = 6
    prof = np.array([1.0, 0.0, 1.0, 1.0, 0.0, 0.0])
    beta = np.broadcast_to(prof[:, None, None], (n, n, n)).copy()
    Ec = sel.culled_moduli(beta)
    nodes = sel.active_nodes(Ec > 0)
    count, label = sel.components(nodes, Ec)
    assert count == 2
    idx = sel.active_dofs(nodes)
    K = fem.assemble(Ec, NU, n)[idx][:, idx].tolil()
    f = fem.load_vectors(Ec, NU, n)[idx]
    for c in range(count):
        first = int(np.flatnonzero(label == c)[0])
        for d in range(3):
            r = 3 * first + d
            K[r, :] = 0.0
            K[:, r] = 0.0
            K[r, r] = 1.0
            f[r] = 0.0
    Ud = spla.splu(K.tocsc()).solve(f)
    U = np.zeros((3 * n ** 3, 6))
    U[idx] = Ud
    C_direct = hom.energy_tensor(Ec, U, NU, n)
    C_cg, _ = sel.homogenize_selective_stiffness(Ec, NU)
    assert np.max(np.abs(C_direct - C_cg)) < 1e-11


def test_full_solid_returns_D():
    n = 4
    C, info = sel.homogenize_selective_stiffness(np.full((n, n, n), 1.7), NU)
    assert np.max(np.abs(C - fem.isotropic_D(1.7, NU))) < 1e-13
    assert info["n_active_nodes"] == n ** 3


def test_active_node_rule_brute_force():
    rng = np.random.default_rng(3)
    n = 4
    act = rng.random((n, n, n)) < 0.15
    got = sel.active_nodes(act)
    want = np.zeros_like(act)
    for k in range(n):
        for j in range(n):
            for i in range(n):
                # voxel (i, j, k) has corners (i + ax, j + ay, k + az) mod n
                if act[k, j, i]:
                    for az in (0, 1):
                        for ay in (0, 1):
                            for ax in (0, 1):
                                want[(k + az) % n, (j + ay) % n, (i + ax) % n] = True
    assert np.array_equal(got, want)
    # the eps rule: beta > 1e-3 strictly
    beta = np.array([0.0, 1e-3, 1.0000001e-3, 0.5]).reshape(1, 1, 4)
    assert sel.active_voxels(beta).ravel().tolist() == [False, False, True, True]


@pytest.mark.parametrize("seed", [11, 12])
def test_dense_floor_tends_to_the_culled_result(seed):
    # hard threshold: the dense oracle with the stiffness floor E_void -> 0
    # approaches the selective result (C^H is monotone in every E_e)
    n = 8
    d = wl.random_design(seed, n, N=8, vf=0.3)
    C_sel, info = sel.homogenize_design_selective(d.pos, d.q, n, target_vf=0.3, nu=NU)
    s = np.abs(C_sel).max()
    prev = None
    for ev in (1e-6, 1e-8, 1e-10):
        C_den, _ = hom.homogenize_design(d.pos, d.q, n, target_vf=0.3, E_void=ev, nu=NU)
        diff = np.abs(C_den - C_sel).max() / s
        # the floor only adds stiffness: C_dense - C_sel is positive semidefinite
        assert np.linalg.eigvalsh(0.5 * (C_den - C_sel + (C_den - C_sel).T)).min() > -1e-10 * s
        if prev is not None:
            assert diff < prev
        prev = diff
    assert prev < 1e-7, prev


def test_octahedral_charges_give_cubic_tensor_and_voigt_bound():
    from test_oracle_homogenize import _gap_threshold
    n = 12
    pos, q = wl.octahedral_orbit(np.array([[0.12, 0.31, 0.07], [0.41, 0.22, 0.36]]), np.array([1.0, -1.0]))
    F, G = fld.field_and_gradient(pos, q, n)
    t = _gap_threshold(fld.distance(F, G), 0.3)
    C, info = sel.homogenize_design_selective(pos, q, n, thickness=t, nu=NU)
    s = np.abs(C).max()
    assert abs(C[0, 0] - C[1, 1]) < 1e-9 * s and abs(C[0, 0] - C[2, 2]) < 1e-9 * s
    assert abs(C[0, 1] - C[0, 2]) < 1e-9 * s and abs(C[0, 1] - C[1, 2]) < 1e-9 * s
    assert abs(C[3, 3] - C[4, 4]) < 1e-9 * s and abs(C[3, 3] - C[5, 5]) < 1e-9 * s
    off = C.copy()
    for i in range(6):
        off[i, i] = 0.0
    off[:3, :3] = 0.0
    assert np.abs(off).max() < 1e-9 * s
    # Voigt: C^H <= <E_e> D (Loewner), with the culled moduli averaged over the cell
    D = fem.isotropic_D(1.0, NU) * info["Ec"].mean()
    assert np.linalg.eigvalsh(D - C).min() > -1e-10 * s


def test_smooth_occupancy_culls_below_eps():
    # logistic occupancy: voxels with beta <= 1e-3 carry nothing, the rest
    # E beta; the culled field through the solve equals a field built by hand
    n = 8
    d = wl.random_design(5, n, N=8, vf=0.3, kappa=32.0)
    F, G = fld.field_and_gradient(d.pos, d.q, n)
    dist = fld.distance(F, G)
    t = fld.thickness_for_volume(dist, 0.3, 32.0)
    beta = fld.occupancy(dist, t, 32.0)
    assert (beta <= 1e-3).any() and (beta > 1e-3).any()
    C, info = sel.homogenize_design_selective(d.pos, d.q, n, thickness=t, kappa=32.0, nu=NU)
    hand = np.where(beta > 1e-3, beta, 0.0)
    assert np.array_equal(info["Ec"], hand)
    C2, _ = sel.homogenize_selective_stiffness(hand, NU)
    assert np.array_equal(C, C2)
    # keeping the sub-eps voxels (no culling) only stiffens
    C_all, _ = hom.homogenize_stiffness(beta, NU)
    assert np.linalg.eigvalsh(C_all - C).min() > -1e-10 * np.abs(C).max()


def test_culled_gradient_matches_finite_differences():
    # brute force: central differences of the culled forward path (field ->
    # logistic shell -> culled solve -> C^H, V) in a few positions and charge
    # values against design_gradient_selective (no voxel crosses eps within h)
    n, kappa = 8, 32.0
    rng = np.random.default_rng(12)
    pos = rng.random((4, 3))
    q = np.array([1.0, -1.0, 0.7, -0.7])
    F, G = fld.field_and_gradient(pos, q, n)
    t = fld.thickness_for_volume(fld.distance(F, G), 0.3, kappa)
    dLdC = rng.standard_normal((6, 6))
    dLdV = -0.4
    C, V, dpos, dq = sel.design_gradient_selective(pos, q, n, dLdC, dLdV, thickness=t, kappa=kappa)

    def loss(p, qq):
        Cp, info = sel.homogenize_design_selective(p, qq, n, thickness=t, kappa=kappa, rtol=1e-13)
        return float(np.sum(dLdC * Cp) + dLdV * info["V"])

    h = 1e-6
    scale = max(np.abs(dpos).max(), np.abs(dq).max())
    for j, c in ((0, 0), (1, 2), (3, 1)):
        pp, pm = pos.copy(), pos.copy()
        pp[j, c] += h
        pm[j, c] -= h
        fd = (loss(pp, q) - loss(pm, q)) / (2 * h)
        assert abs(fd - dpos[j, c]) <= 2e-5 * scale, (j, c, fd, dpos[j, c])
    for j in (0, 2):
        qp, qm = q.copy(), q.copy()
        qp[j] += h
        qm[j] -= h
        fd = (loss(pos, qp) - loss(pos, qm)) / (2 * h)
        assert abs(fd - dq[j]) <= 2e-5 * scale, (j, fd, dq[j])
