"""End-to-end parity of the HIP path with the oracle and the closed forms."""
import json
import os

import numpy as np
import pytest

from gpu_helpers import assert_ch_close, torch
from oracle import fem, homogenize as hom
from paper_2511_04025_amd import workloads as wl

pytestmark = pytest.mark.gpu


def api():
    from paper_2511_04025_amd import api as A
    return A


def test_full_solid_and_laminate_closed_forms():
    A = api()
    n = 16
    for prec in ("fp64", "mixed"):
        r = A.homogenize_stiffness(torch.full((n, n, n), 2.0, dtype=torch.float64, device="cuda"), 0.3,
                                   precision=prec)
        assert np.max(np.abs(r["C"] - fem.isotropic_D(2.0, 0.3))) <= 1e-12 * 2.0
        assert r["status"] == 0
    # z laminate of whole voxel layers: Backus averages (exact in the trilinear space)
    E = np.full((n, n, n), 1e-3)
    E[: n // 4] = 1.0
    E[n // 2: n // 2 + 2] = 0.4
    from test_oracle_homogenize import backus_z
    phases = []
    for e in sorted(set(E[:, 0, 0])):
        lam, mu = fem.lame(e, 0.3)
        phases.append((np.mean(E[:, 0, 0] == e), lam, mu))
    ref = backus_z(phases)
    for prec, tol in (("fp64", 1e-8), ("mixed", 1e-5)):
        r = A.homogenize_stiffness(torch.tensor(E, device="cuda"), 0.3, precision=prec,
                                   rtol=1e-11 if prec == "fp64" else 1e-7)
        assert np.max(np.abs(r["C"] - ref)) <= tol * np.abs(ref).max(), prec


@pytest.mark.parametrize("n,seed", [(12, 1), (20, 2)])
def test_fp64_path_matches_oracle_small(n, seed):
    A = api()
    d = wl.random_design(seed, n, N=12, vf=0.2, E_void=1e-3)
    C, info = hom.homogenize_design(d.pos, d.q, n, target_vf=d.target_vf, E_void=d.E_void)
    r = A.homogenize(d, precision="fp64", rtol=1e-11)
    assert r["status"] == 0
    assert r["V"] == info["V"]
    assert_ch_close(r["C"], C, 1e-8)
    assert np.all(r["rel_res"] <= 1e-11)


def golden(name):
    with open(os.path.join(os.path.dirname(__file__), "golden", name)) as f:
        return json.load(f)


def test_small_shell_fp64_vs_oracle():
    # 24^3, 16 charges of +-1, V = 0.12, void E = 1e-3, FP64 PCG to 1e-10
    A = api()
    g = golden("small_shell_n24_seed1.json")
    r = A.homogenize(wl.small_shell_24(), precision="fp64", rtol=1e-10)
    assert r["status"] == 0 and np.all(r["rel_res"] <= 1e-10)
    assert r["V"] == g["V"]
    assert abs(r["t"] - g["t"]) <= 1e-12 * g["t"]
    assert_ch_close(r["C"], np.array(g["C"]), 1e-7)


@pytest.mark.parametrize("precision,tol", [("mixed", 1e-4), ("fp64", 1e-7)])
def test_small_shell_mixed_and_fp64(precision, tol):
    A = api()
    g = golden("small_shell_n24_seed1.json")
    r = A.homogenize(wl.small_shell_24(), precision=precision)
    assert r["status"] == 0
    assert_ch_close(r["C"], np.array(g["C"]), tol)


@pytest.mark.parametrize("n,seed", [(16, 3), (20, 4)])
def test_mixed_path_matches_oracle(n, seed):
    A = api()
    d = wl.random_design(seed, n, N=16, vf=0.12, E_void=1e-3, pm=False)
    C, info = hom.homogenize_design(d.pos, d.q, n, target_vf=d.target_vf, E_void=d.E_void)
    r = A.homogenize(d, precision="mixed", rtol=1e-6)
    assert r["status"] == 0
    assert r["V"] == info["V"]
    assert_ch_close(r["C"], C, 1e-4)


@pytest.mark.parametrize("seed", [5000, 5001])
@pytest.mark.parametrize("precision,tol", [("mixed", 1e-4), ("fp64", 1e-7)])
def test_logistic_void_1e6_vs_golden(seed, precision, tol):
    # 24^3, 32 charges of +-1, logistic occupancy (kappa = 4n), void E = 1e-6
    A = api()
    g = golden(f"smooth_shell_n24_seed{seed}.json")
    d = wl.smooth_shell_96(seed, n=24).with_(thickness=g["t"])
    r = A.homogenize(d, precision=precision)
    assert r["status"] == 0
    assert abs(r["V"] - g["V"]) <= 1e-13
    assert_ch_close(r["C"], np.array(g["C"]), tol)


@pytest.mark.parametrize("solver,n", [("jacobi", 14), ("mg", 16)])
def test_field_entry_point_encodings_vs_oracle(solver, n):
    # shh_homogenize_field in its three encodings of the same hard-threshold
    # shell: the 1-byte solid/void code (E, E_void rebuilt in the kernel),
    # FP32 moduli and FP64 moduli, each against the oracle's C^H of exactly
    # the moduli the encoding carries (FP64 solve to 1e-11, bar 1e-8; mixed
    # at 1e-7, bar 1e-4)
    from oracle import field as fld
    A = api()
    d = wl.random_design(77 + n, n, N=12, vf=0.2)
    F, G = fld.field_and_gradient(d.pos, d.q, n)
    dist = fld.distance(F, G)
    beta = fld.occupancy(dist, fld.thickness_for_volume(dist, 0.2, 0.0), 0.0)
    Es, Ev, nu = 1.3, 2e-3, 0.3
    E64 = fld.stiffness_field(beta, Es, Ev)
    E32 = E64.astype(np.float32)
    cases = {"u8": (torch.tensor(beta.astype(np.uint8), device="cuda"), E64, beta.mean()),
             "f32": (torch.tensor(E32, device="cuda"), E32.astype(np.float64), None),
             "f64": (torch.tensor(E64, device="cuda"), E64, None)}
    for name, (grid, ref_E, V) in cases.items():
        C_ref, _ = hom.homogenize_stiffness(ref_E, nu, solver="direct")
        for prec, rtol, tol in (("fp64", 1e-11, 1e-8), ("mixed", 1e-7, 1e-4)):
            r = A.homogenize_field(grid, nu, E_solid=Es, E_void=Ev, precision=prec, rtol=rtol, solver=solver)
            assert r["status"] == 0, (name, prec)
            assert_ch_close(r["C"], C_ref, tol)
            if V is not None:
                assert r["V"] == V
            else:
                assert abs(r["V"] - ref_E.mean() / ref_E.max()) <= 1e-14
