"""Pins of the oracle's homogenized tensor C^H (Eq. (8)).

Closed forms: a fully solid cell returns the base isotropic tensor; whole-voxel
laminates return the Backus averages (Reuss across the layers, Voigt along
them), which the trilinear element reproduces exactly.  Invariants: symmetry,
positive definiteness, the Voigt and Reuss Loewner bounds, cubic symmetry of
octahedral charge sets, the axis-swap permutation, whole-voxel translations,
1-homogeneity in E, the Hashin-Shtrikman bulk bound, and agreement of the
energy and mixed forms and of CG with a direct solve.
"""
import numpy as np
import pytest

from oracle import fem, field as fld, homogenize as hom, metrics
from paper_2511_04025_amd import workloads as wl

NU = 0.3


def backus_z(phases):
    """Closed-form effective tensor of isotropic layers stacked along z.
    phases: list of (volume fraction, lambda, mu)."""
    f = np.array([p[0] for p in phases])
    lam = np.array([p[1] for p in phases])
    mu = np.array([p[2] for p in phases])
    P = lam + 2 * mu
    avg = lambda v: np.sum(f * v)
    C33 = 1.0 / avg(1.0 / P)
    r = avg(lam / P)
    C = np.zeros((6, 6))
    C[2, 2] = C33
    C[0, 2] = C[2, 0] = C[1, 2] = C[2, 1] = r * C33
    C[0, 0] = C[1, 1] = avg(P - lam ** 2 / P) + r * r * C33
    C[0, 1] = C[1, 0] = avg(lam - lam ** 2 / P) + r * r * C33
    C[3, 3] = C[4, 4] = 1.0 / avg(1.0 / mu)
    C[5, 5] = avg(mu)
    return C


# Voigt index permutation for relabelling axes: new axis a = old axis perm[a]
def voigt_perm(perm):
    pairs = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]
    idx = []
    for (a, b) in pairs:
        oa, ob = sorted((perm[a], perm[b]))
        idx.append(pairs.index((oa, ob)))
    return np.array(idx)


def test_full_solid_returns_D():
    n = 5
    C, info = hom.homogenize_stiffness(np.full((n, n, n), 2.5), NU)
    assert np.max(np.abs(C - fem.isotropic_D(2.5, NU))) < 1e-13
    # the load vectors are zero up to rounding, so u stays at rounding level
    assert np.max(np.abs(info["U"])) < 1e-12


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_laminate_backus(axis):
    n = 6
    moduli = [1.0, 1.0, 0.3, 1e-3, 1e-3, 0.3]  # layers along the chosen axis
    Ee = np.zeros((n, n, n))
    for layer, e in enumerate(moduli):
        if axis == 2:
            Ee[layer, :, :] = e
        elif axis == 1:
            Ee[:, layer, :] = e
        else:
            Ee[:, :, layer] = e
    C, info = hom.homogenize_stiffness(Ee, NU, solver="direct")
    phases = []
    for e in sorted(set(moduli)):
        lam, mu = fem.lame(e, NU)
        phases.append((moduli.count(e) / n, lam, mu))
    Cz = backus_z(phases)
    # relabel: the stacking axis plays the role of z
    perm = {2: (0, 1, 2), 1: (0, 2, 1), 0: (2, 1, 0)}[axis]
    p = voigt_perm(perm)
    ref = Cz[np.ix_(p, p)]
    assert np.max(np.abs(C - ref)) < 1e-12
    # the Voigt bound <E> on the in-plane Young's modulus of a z laminate
    if axis == 2:
        assert metrics.young_moduli(C)[0] <= np.mean(moduli) + 1e-12


def _design_C(d, n, **kw):
    return hom.homogenize_design(d.pos, d.q, n, target_vf=d.target_vf, E_void=d.E_void,
                                 kappa=d.kappa, **kw)


def test_symmetry_definiteness_and_loewner_bounds():
    d = wl.random_design(31, 10, N=12, vf=0.25, E_void=1e-2)
    C, info = _design_C(d, 10, solver="direct")
    assert np.max(np.abs(C - C.T)) < 1e-12 * np.abs(C).max()
    assert np.min(np.linalg.eigvalsh(C)) > 0
    Ee = info["Ee"]
    D1 = fem.isotropic_D(1.0, NU)
    voigt = Ee.mean() * D1
    reuss = D1 / np.mean(1.0 / Ee)
    assert np.max(np.linalg.eigvalsh(C - voigt)) < 1e-12
    assert np.min(np.linalg.eigvalsh(C - reuss)) > -1e-12
    # energy and mixed forms agree at equilibrium
    Cm = hom.mixed_form_tensor(Ee, info["U"], NU, 10)
    assert np.max(np.abs(C - Cm)) < 1e-10 * np.abs(C).max()


def test_cg_and_direct_agree_on_CH():
    d = wl.random_design(32, 8, N=10, vf=0.3, E_void=1e-3)
    C1, i1 = _design_C(d, 8, solver="cg", rtol=1e-12)
    C2, _ = _design_C(d, 8, solver="direct")
    assert np.max(np.abs(C1 - C2)) < 1e-11 * np.abs(C2).max()
    assert np.all(i1["rel_res"] < 2e-12)


def _gap_threshold(dist, vf):
    """A thickness inside a clear gap of the sorted distances near vf, so that
    voxels related by symmetry (equal d up to rounding) fall on one side."""
    s = np.sort(dist.ravel())
    k = int(vf * s.size)
    for off in range(s.size):
        for kk in (k + off, k - off):
            if 1 <= kk < s.size and s[kk] - s[kk - 1] > 1e-9 * s[-1]:
                return 0.5 * (s[kk] + s[kk - 1])
    raise AssertionError("no gap")


def test_octahedral_charges_give_cubic_tensor_and_hs_bound():
    p, q = wl.octahedral_orbit(np.array([[0.12, 0.31, 0.07], [0.41, 0.22, 0.36]]), np.array([1.0, -1.0]))
    assert len(q) == 96
    n = 12
    F, G = fld.field_and_gradient(p, q, n)
    dist = fld.distance(F, G)
    t = _gap_threshold(dist, 0.3)
    C, info = hom.homogenize_design(p, q, n, thickness=t, E_void=1e-3, solver="direct")
    s = np.abs(C).max()
    tol = 1e-10 * s
    assert abs(C[0, 0] - C[1, 1]) < tol and abs(C[0, 0] - C[2, 2]) < tol
    assert abs(C[0, 1] - C[0, 2]) < tol and abs(C[0, 1] - C[1, 2]) < tol
    assert abs(C[3, 3] - C[4, 4]) < tol and abs(C[3, 3] - C[5, 5]) < tol
    mask = np.ones((6, 6), bool)
    mask[:3, :3] = False
    for i in range(3, 6):
        mask[i, i] = False
    assert np.max(np.abs(C[mask])) < tol
    # Hashin-Shtrikman upper bound on the bulk modulus (cubic => isotropic bulk response)
    V = info["V"]
    K1, G1 = fem.lame(1.0, NU)[0] + 2.0 / 3.0 * fem.lame(1.0, NU)[1], fem.lame(1.0, NU)[1]
    lv, mv = fem.lame(1e-3, NU)
    KU, GU = metrics.hashin_shtrikman_upper(V, K1, G1, lv + 2.0 / 3.0 * mv, mv)
    Kc = (C[0, 0] + 2 * C[0, 1]) / 3.0
    assert 0 < Kc <= KU


def test_mirror_charges_give_orthotropic_tensor():
    p, q = wl.mirror_orbit(np.array([[0.13, 0.29, 0.41], [0.37, 0.08, 0.19]]), np.array([1.0, -1.0]))
    n = 10
    F, G = fld.field_and_gradient(p, q, n)
    t = _gap_threshold(fld.distance(F, G), 0.3)
    C, _ = hom.homogenize_design(p, q, n, thickness=t, E_void=1e-3, solver="direct")
    tol = 1e-10 * np.abs(C).max()
    assert np.max(np.abs(C[:3, 3:])) < tol
    assert abs(C[3, 4]) < tol and abs(C[3, 5]) < tol and abs(C[4, 5]) < tol


def test_axis_swap_permutes_tensor_and_voxel_shift_invariance():
    d = wl.random_design(33, 8, N=10, vf=0.3, E_void=1e-3)
    n = 8
    C, info = _design_C(d, n, solver="direct")
    t = info["t"]
    swapped = d.pos[:, [1, 0, 2]]
    C2, _ = hom.homogenize_design(swapped, d.q, n, thickness=t, E_void=d.E_void, solver="direct")
    p = voigt_perm((1, 0, 2))
    assert np.max(np.abs(C2 - C[np.ix_(p, p)])) < 1e-10 * np.abs(C).max()
    C3, _ = hom.homogenize_design(d.pos + np.array([1.0 / n, 3.0 / n, 0.0]), d.q, n, thickness=t,
                                  E_void=d.E_void, solver="direct")
    assert np.max(np.abs(C3 - C)) < 1e-10 * np.abs(C).max()
    # 1-homogeneity in the moduli
    C4, _ = hom.homogenize_design(d.pos, d.q, n, thickness=t, E=3.0, E_void=3.0 * d.E_void, solver="direct")
    assert np.max(np.abs(C4 - 3.0 * C)) < 1e-10 * np.abs(C).max()


def test_design_path_moduli_full_solid():
    """Through the whole forward path: a half-thickness above every distance
    makes every voxel solid, so C^H = E D exactly (E_void plays no part)."""
    d = wl.random_design(11, 6, N=8, pm=True)
    C, info = hom.homogenize_design(d.pos, d.q, 6, thickness=1e300, E=2.5, E_void=0.1, nu=NU)
    assert info["V"] == 1.0
    assert np.max(np.abs(C - fem.isotropic_D(2.5, NU))) < 1e-13 * 2.5


def test_design_path_moduli_planar_field_backus():
    """Through the whole forward path: a field of (0,0,l) modes only gives whole
    voxel layers, solid ones at E and void ones at the floor E_void, so C^H is
    the Backus laminate of those two moduli -- which fixes the modulus mapping
    E_e = E_void + (E - E_void) beta_e voxel by voxel."""
    d = wl.random_design(5, 8, N=8, pm=True)
    alpha = np.zeros((4, 4, 4))
    alpha[0, 0, 1] = 1.0
    alpha[0, 0, 3] = 0.4
    n, E, Ev = 8, 1.7, 0.05
    C, info = hom.homogenize_design(d.pos, d.q, n, alpha=alpha, target_vf=0.5, E=E, E_void=Ev,
                                    nu=NU, solver="direct")
    assert info["V"] == 0.5
    phases = []
    for e in (E, Ev):
        lam, mu = fem.lame(e, NU)
        phases.append((0.5, lam, mu))
    assert np.max(np.abs(C - backus_z(phases))) < 1e-12
