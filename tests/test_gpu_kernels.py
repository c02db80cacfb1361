"""Per-step parity of the HIP path against the FP64 oracle on seeded inputs.

Sizes span several stencil tiles (32 x 8 x 16) and ragged tails (n = 20, 37),
plus the degenerate n = 2 and n = 3 grids where the periodic halo wraps onto
the tile itself.
"""
import numpy as np
import pytest

from gpu_helpers import nodal_to_oracle, oracle_to_nodal, torch
from oracle import fem, field as fld
from paper_2511_04025_amd import workloads as wl

pytestmark = pytest.mark.gpu


def api():
    from paper_2511_04025_amd import api as A
    return A


@pytest.mark.parametrize("n,N,K", [(20, 16, 3), (37, 9, 2), (3, 4, 3), (64, 24, 3)])
def test_field_distance_occupancy(n, N, K):
    A = api()
    d = wl.random_design(100 + n, n, N=N, vf=0.15, pm=False).with_(K=K)
    F, G = fld.field_and_gradient(d.pos, d.q, n, K=K)
    dist = fld.distance(F, G)
    t = fld.thickness_for_volume(dist, 0.15, 0.0)
    out = A.field(d.with_(thickness=t))
    Fg, Gg, dg, bg = (out[k].cpu().numpy() for k in ("F", "G", "d", "beta"))
    sF = np.abs(F).max()
    assert np.max(np.abs(Fg - F)) <= 1e-13 * sF
    assert np.max(np.abs(Gg - G)) <= 1e-13 * np.abs(G).max()
    assert np.max(np.abs(dg - dist)) <= 1e-11 * dist.max()
    beta = fld.occupancy(dist, t, 0.0)
    assert np.array_equal(bg, beta)  # the hard step decides voxel for voxel
    assert out["V"] == beta.mean()


def test_alpha_weights_and_dist_mode1():
    A = api()
    n = 16
    d = wl.random_design(7, n, N=10, pm=True)
    rng = np.random.default_rng(3)
    alpha = rng.uniform(0.2, 1.5, (4, 4, 4))
    F, G = fld.field_and_gradient(d.pos, d.q, n, alpha=alpha)
    out = A.field(d.with_(alpha=alpha, thickness=0.05, dist_mode=1, iso=0.01))
    assert np.max(np.abs(out["F"].cpu().numpy() - F)) <= 1e-13 * np.abs(F).max()
    assert np.max(np.abs(out["d"].cpu().numpy() - np.abs(F - 0.01))) <= 1e-13 * np.abs(F).max()


@pytest.mark.parametrize("vf", [0.03, 0.12, 0.2])
def test_hard_thickness_selection_matches_oracle(vf):
    A = api()
    n = 24
    d = wl.random_design(55, n, N=16, vf=vf)
    F, G = fld.field_and_gradient(d.pos, d.q, n)
    dist = fld.distance(F, G)
    t = fld.thickness_for_volume(dist, vf, 0.0)
    out = A.field(d)  # GPU chooses t itself
    beta = fld.occupancy(dist, t, 0.0)
    assert np.array_equal(out["beta"].cpu().numpy(), beta)
    assert abs(out["t"] - t) <= 1e-12 * t
    assert int(beta.sum()) == int(np.floor(vf * n ** 3 + 0.5))


def test_logistic_thickness_bisection():
    A = api()
    n = 20
    d = wl.random_design(56, n, N=16, vf=0.1, kappa=4.0 * n)
    out = A.field(d)
    assert abs(out["V"] - 0.1) <= 1e-12
    F, G = fld.field_and_gradient(d.pos, d.q, n)
    dist = fld.distance(F, G)
    t = fld.thickness_for_volume(dist, 0.1, 4.0 * n)
    assert abs(out["t"] - t) <= 1e-9


def _moduli(n, seed, contrast=1e-3):
    rng = np.random.default_rng(seed)
    return np.where(rng.random((n, n, n)) < 0.35, 1.0, contrast) * rng.uniform(0.5, 1.0, (n, n, n))


@pytest.mark.parametrize("n", [2, 3, 20, 37])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_stiffness_operator_matches_assembled_matrix(n, precision):
    A = api()
    nu = 0.3
    E = _moduli(n, n)
    K = fem.assemble(E, nu, n)
    rng = np.random.default_rng(11)
    U = rng.standard_normal((3 * n ** 3, 6))
    Q = K @ U
    dt = torch.float64 if precision == "fp64" else torch.float32
    p = torch.tensor(oracle_to_nodal(U, n), dtype=dt, device="cuda")
    q = A.apply_stiffness(torch.tensor(E, device="cuda"), p, nu, precision)
    Qg = nodal_to_oracle(q.double().cpu().numpy(), n)
    tol = 1e-13 if precision == "fp64" else 2e-6
    assert np.max(np.abs(Qg - Q)) <= tol * np.abs(Q).max()


def test_stiffness_operator_poisson_ratios():
    A = api()
    n = 9
    E = _moduli(n, 5)
    rng = np.random.default_rng(12)
    U = rng.standard_normal((3 * n ** 3, 6))
    for nu in (-0.5, 0.0, 0.45):
        Q = fem.assemble(E, nu, n) @ U
        q = A.apply_stiffness(torch.tensor(E, device="cuda"),
                              torch.tensor(oracle_to_nodal(U, n), device="cuda"), nu, "fp64")
        assert np.max(np.abs(nodal_to_oracle(q.cpu().numpy(), n) - Q)) <= 1e-13 * np.abs(Q).max()


@pytest.mark.parametrize("n", [3, 20])
def test_load_vectors(n):
    A = api()
    E = _moduli(n, 21)
    f = fem.load_vectors(E, 0.3, n)
    fg = A.load_vectors(torch.tensor(E, device="cuda"), 0.3)
    assert np.max(np.abs(nodal_to_oracle(fg.cpu().numpy(), n) - f)) <= 1e-13 * np.abs(f).max()


@pytest.mark.parametrize("n", [3, 20])
def test_energy_form(n):
    A = api()
    from oracle import homogenize as hom
    E = _moduli(n, 22)
    rng = np.random.default_rng(2)
    U = 0.1 * rng.standard_normal((3 * n ** 3, 6))
    C = hom.energy_tensor(E, U, 0.3, n)
    Cg = A.energy(torch.tensor(E, device="cuda"), torch.tensor(oracle_to_nodal(U, n), device="cuda"), 0.3)
    assert np.max(np.abs(Cg - C)) <= 1e-13 * np.abs(C).max()
