"""Pins of the oracle's field, distance, occupancy and thickness rule.

Each test checks the oracle against something other than its own formula:
closed forms (the Dirichlet kernel, a single cosine mode, the Schwarz-P-like
two-charge cell), calculus (central differences), symmetries (lattice
periodicity, whole-voxel translations, charge scaling) and exact counts.
"""
import numpy as np
import pytest

from oracle import field as fld
from paper_2511_04025_amd import workloads as wl


def dirichlet(K, s):
    """D_K(s) = sum_{m=-K..K} exp(2 pi i m s) = sin((2K+1) pi s) / sin(pi s)."""
    s = np.asarray(s, dtype=np.float64)
    out = np.empty_like(s)
    small = np.abs(np.sin(np.pi * s)) < 1e-12
    out[~small] = np.sin((2 * K + 1) * np.pi * s[~small]) / np.sin(np.pi * s[~small])
    out[small] = 2 * K + 1
    return out


@pytest.mark.parametrize("K", [1, 2, 3, 4])
def test_weights_against_dirichlet_kernel(K):
    # alpha_hkl = h^2+k^2+l^2 cancels the 1/(h^2+k^2+l^2) factor of Eq. (6); with
    # one unit charge at the origin the octant sum with weights w_hkl is the
    # product of three Dirichlet kernels: 8 (F + 1/8) = D_K(x) D_K(y) D_K(z).
    alpha = np.zeros((K + 1,) * 3)
    for h in range(K + 1):
        for k in range(K + 1):
            for l in range(K + 1):
                alpha[h, k, l] = h * h + k * k + l * l
    rng = np.random.default_rng(7)
    pts = rng.random((200, 3))
    F = fld.field_at_points(pts, np.zeros((1, 3)), np.ones(1), K=K, alpha=alpha)
    ref = dirichlet(K, pts[:, 0]) * dirichlet(K, pts[:, 1]) * dirichlet(K, pts[:, 2]) / 8.0 - 1.0 / 8.0
    assert np.max(np.abs(F - ref)) < 1e-12
    n = 8
    Fg, _ = fld.field_and_gradient(np.zeros((1, 3)), np.ones(1), n, K=K, alpha=alpha)
    c = fld.voxel_centers(n)
    refg = (dirichlet(K, c)[:, None, None] * dirichlet(K, c)[None, :, None]
            * dirichlet(K, c)[None, None, :]) / 8.0 - 1.0 / 8.0
    assert np.max(np.abs(Fg - refg)) < 1e-12


def test_single_mode_closed_form():
    # only alpha_100 = 1: w_100 = 1/4 and h^2+k^2+l^2 = 1, so
    # F = (1/4) sum_j q_j cos(2 pi (x - x_j)).
    alpha = np.zeros((4, 4, 4))
    alpha[1, 0, 0] = 1.0
    pos = np.array([[0.1, 0.7, 0.3], [0.55, 0.2, 0.9]])
    q = np.array([1.0, -1.0])
    n = 10
    F, G = fld.field_and_gradient(pos, q, n, K=3, alpha=alpha)
    x = fld.voxel_centers(n)
    ref = 0.25 * (np.cos(2 * np.pi * (x - 0.1)) - np.cos(2 * np.pi * (x - 0.55)))
    assert np.max(np.abs(F - ref[None, None, :])) < 1e-14
    dref = -0.5 * np.pi * (np.sin(2 * np.pi * (x - 0.1)) - np.sin(2 * np.pi * (x - 0.55)))
    assert np.max(np.abs(G[0] - dref[None, None, :])) < 1e-13
    assert np.max(np.abs(G[1])) == 0.0 and np.max(np.abs(G[2])) == 0.0


def test_schwarz_p_like_coefficients():
    # +1 at the origin, -1 at the body center: cos(2 pi h (x - 1/2)) = (-1)^h cos(2 pi h x),
    # so only modes with h+k+l odd survive, each with 2 w_hkl / (h^2+k^2+l^2).
    # Hand values: (1,0,0): 2*(1/4)/1 = 1/2 (the P-surface nodal approximation
    # (cos 2pi x + cos 2pi y + cos 2pi z)/2); (1,1,1): 2/3; (2,1,0): 1/5;
    # (3,0,0): 1/18; (2,2,1): 2/9; even modes vanish.
    pos = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.5]])
    q = np.array([1.0, -1.0])
    n = 16
    F, _ = fld.field_and_gradient(pos, q, n, K=3)
    c = fld.voxel_centers(n)

    def coeff(h, k, l):
        b = (np.cos(2 * np.pi * l * c)[:, None, None] * np.cos(2 * np.pi * k * c)[None, :, None]
             * np.cos(2 * np.pi * h * c)[None, None, :])
        return np.sum(F * b) / np.sum(b * b)

    expected = {(1, 0, 0): 0.5, (0, 1, 0): 0.5, (0, 0, 1): 0.5, (1, 1, 1): 2.0 / 3.0,
                (2, 1, 0): 0.2, (0, 1, 2): 0.2, (3, 0, 0): 1.0 / 18.0, (2, 2, 1): 2.0 / 9.0,
                (2, 0, 0): 0.0, (1, 1, 0): 0.0, (2, 2, 0): 0.0, (3, 1, 0): 0.0}
    for mode, val in expected.items():
        assert abs(coeff(*mode) - val) < 1e-12, mode
    # symmetric under axis permutations
    assert np.max(np.abs(F - F.transpose(1, 0, 2))) < 1e-13
    assert np.max(np.abs(F - F.transpose(2, 1, 0))) < 1e-13


def test_gradient_central_differences():
    d = wl.random_design(3, 6, N=6, pm=False)
    n = 6
    F, G = fld.field_and_gradient(d.pos, d.q, n)
    c = fld.voxel_centers(n)
    kk, jj, ii = np.meshgrid(c, c, c, indexing="ij")
    pts = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1)
    h = 1e-5
    for ax in range(3):
        e = np.zeros(3)
        e[ax] = h
        fd = (fld.field_at_points(pts + e, d.pos, d.q) - fld.field_at_points(pts - e, d.pos, d.q)) / (2 * h)
        scale = np.abs(G[ax]).max()
        assert np.max(np.abs(fd - G[ax].ravel())) < 1e-7 * scale
    assert np.max(np.abs(fld.field_at_points(pts, d.pos, d.q) - F.ravel())) < 1e-13


def test_lattice_periodicity_and_voxel_translation():
    d = wl.random_design(11, 8, N=8, pm=True)
    n = 8
    F, G = fld.field_and_gradient(d.pos, d.q, n)
    shifted = d.pos + np.array([[1.0, -2.0, 3.0]] * len(d.q))
    F2, _ = fld.field_and_gradient(shifted, d.q, n)
    assert np.max(np.abs(F - F2)) < 1e-12
    # moving every charge by whole voxels (2/n in x, 1/n in z) rolls the grid
    F3, G3 = fld.field_and_gradient(d.pos + np.array([2.0 / n, 0.0, 1.0 / n]), d.q, n)
    assert np.max(np.abs(F3 - np.roll(F, (1, 0, 2), axis=(0, 1, 2)))) < 1e-12
    assert np.max(np.abs(G3 - np.roll(G, (1, 0, 2), axis=(1, 2, 3)))) < 1e-11


def test_distance_invariant_to_charge_scale_and_planar_volume():
    d = wl.random_design(5, 10, N=8, pm=True)
    F, G = fld.field_and_gradient(d.pos, d.q, 10)
    F2, G2 = fld.field_and_gradient(d.pos, 3.7 * d.q, 10)
    d1 = fld.distance(F, G)
    d2 = fld.distance(F2, G2)
    assert np.max(np.abs(d1 - d2)) < 1e-12 * max(1.0, d1.max())
    # a field built only from (0,0,l) modes depends on z alone, so the hard
    # shell is a stack of whole voxel layers and V = (solid layers) / n exactly
    alpha = np.zeros((4, 4, 4))
    alpha[0, 0, 1] = 1.0
    alpha[0, 0, 3] = 0.4
    n = 12
    Fp, Gp = fld.field_and_gradient(d.pos, d.q, n, alpha=alpha)
    dp = fld.distance(Fp, Gp)
    assert np.max(np.abs(dp - dp[:, :1, :1])) < 1e-12
    t = 0.5 * (np.sort(dp[:, 0, 0])[3] + np.sort(dp[:, 0, 0])[4])
    beta = fld.occupancy(dp, t, 0.0)
    assert beta.mean() == 4.0 / n


def test_distance_mode1_and_floor():
    F = np.array([[[0.0, 0.5]]])
    G = np.zeros((3, 1, 1, 2))
    G[0, 0, 0, 1] = 2.0
    assert np.allclose(fld.distance(F, G), [[[0.0, 0.25]]])
    assert np.allclose(fld.distance(F - 0.1, G, iso=-0.1), [[[0.0, 0.25]]])
    assert np.allclose(fld.distance(F, G, dist_mode=1), [[[0.0, 0.5]]])


@pytest.mark.parametrize("vf", [0.05, 0.12, 0.3])
def test_thickness_for_volume_hard_counts(vf):
    d = wl.random_design(21, 12, N=16)
    F, G = fld.field_and_gradient(d.pos, d.q, 12)
    dist = fld.distance(F, G)
    t = fld.thickness_for_volume(dist, vf, 0.0)
    beta = fld.occupancy(dist, t, 0.0)
    k = int(np.floor(vf * 12 ** 3 + 0.5))
    assert int(beta.sum()) == k
    # idempotent: asking for the volume just obtained returns the same t
    assert fld.thickness_for_volume(dist, beta.mean(), 0.0) == t


def test_thickness_for_volume_logistic():
    d = wl.random_design(22, 10, N=16)
    F, G = fld.field_and_gradient(d.pos, d.q, 10)
    dist = fld.distance(F, G)
    kappa = 40.0
    t = fld.thickness_for_volume(dist, 0.1, kappa)
    assert abs(fld.occupancy(dist, t, kappa).mean() - 0.1) <= 1e-12
    assert fld.occupancy(np.array([t]), t, kappa)[0] == 0.5
    # logistic tends to the hard step as kappa grows
    assert np.all(fld.occupancy(np.array([t - 0.1, t + 0.1]), t, 1e4) == np.array([1.0, 0.0]))


def test_point_evaluation_matches_grid():
    d = wl.random_design(12, 7, N=6, pm=False)
    n = 7
    F, G = fld.field_and_gradient(d.pos, d.q, n)
    c = fld.voxel_centers(n)
    rng = np.random.default_rng(4)
    idx = rng.integers(0, n, (30, 3))  # (i, j, k)
    pts = np.stack([c[idx[:, 0]], c[idx[:, 1]], c[idx[:, 2]]], axis=1)
    Fp, Gp = fld.field_and_gradient_at_points(pts, d.pos, d.q)
    assert np.max(np.abs(Fp - F[idx[:, 2], idx[:, 1], idx[:, 0]])) < 1e-13
    for ax in range(3):
        assert np.max(np.abs(Gp[:, ax] - G[ax][idx[:, 2], idx[:, 1], idx[:, 0]])) < 1e-12
    assert np.max(np.abs(Fp - fld.field_at_points(pts, d.pos, d.q))) < 1e-13
