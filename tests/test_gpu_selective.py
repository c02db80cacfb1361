"""The selective (active-set) solve of Sec. 4.2 on compact node lists
with either preconditioner (solver="selective": the multigrid V-cycle on the
culled hierarchy; "selective-jacobi"): C^H against the culled oracle -- stored
values at 24^3 and 48^3, the free-plate closed form, a fully solid and an
empty cell -- in FP64 and in the mixed path, and the active-node count against
the oracle's."""
import json
import os

import numpy as np
import pytest

from gpu_helpers import assert_ch_close, ch_errors, torch
from paper_2511_04025_amd import workloads as wl

pytestmark = pytest.mark.gpu


def golden(name):
    with open(os.path.join(os.path.dirname(__file__), "golden", name)) as f:
        return json.load(f)


def api():
    from paper_2511_04025_amd import api as A
    return A


SOLVERS = ["selective", "selective-jacobi"]


@pytest.mark.parametrize("solver", SOLVERS)
@pytest.mark.parametrize("precision,rtol,tol", [("fp64", 1e-11, 1e-7), ("mixed", 3e-6, 1e-4)])
def test_small_shell_vs_culled_oracle(precision, rtol, tol, solver):
    A = api()
    g = golden("selective_n24_seed1.json")
    print(f"{solver} 24^3 {precision}", flush=True)
    r = A.homogenize(wl.small_shell_24(), precision=precision, rtol=rtol, solver=solver)
    print("selective iters", r["iters"], "active nodes", r["active_nodes"], flush=True)
    assert r["status"] == 0 and np.all(r["rel_res"] <= rtol)
    assert r["V"] == g["V"] and r["active_nodes"] == g["active_nodes"]
    assert_ch_close(r["C"], np.array(g["C"]), tol)


@pytest.mark.parametrize("solver", SOLVERS)
@pytest.mark.parametrize("precision,rtol,tol", [("fp64", 1e-11, 1e-7), ("mixed", 3e-6, 1e-4)])
def test_shell_designs_at_48_vs_culled_oracle(precision, rtol, tol, solver):
    A = api()
    for seed in (2000, 2001, 2002, 2003):
        g = golden(f"selective_n48_seed{seed}.json")
        d = wl.shell_128(seed, n=48)
        print(f"{solver} 48^3 seed {seed} {precision}", flush=True)
        r = A.homogenize(d, precision=precision, rtol=rtol, solver=solver)
        rel, small, frob = ch_errors(r["C"], np.array(g["C"]))
        print(f"  iters {r['iters'].tolist()} active nodes {r['active_nodes']} ({r['active_nodes'] / 48 ** 3:.3f}) "
              f"rel {rel:.2e} small {small:.2e}", flush=True)
        assert r["status"] == 0 and r["V"] == g["V"] and r["active_nodes"] == g["active_nodes"]
        assert_ch_close(r["C"], np.array(g["C"]), tol)


@pytest.mark.parametrize("solver", SOLVERS)
def test_logistic_design_culls_below_eps(solver):
    A = api()
    g = golden("selective_n24_seed5000.json")
    d = wl.smooth_shell_96(5000, n=24).with_(thickness=g["t"])
    r = A.homogenize(d, precision="fp64", rtol=1e-11, solver=solver)
    assert r["status"] == 0 and abs(r["V"] - g["V"]) <= 1e-13
    assert r["active_nodes"] == g["active_nodes"]
    assert_ch_close(r["C"], np.array(g["C"]), 1e-7)


def _plate(fs, nu=0.3, axis=2):
    lam = nu / ((1 + nu) * (1 - 2 * nu))
    mu = 1.0 / (2 * (1 + nu))
    P = lam + 2 * mu
    C = np.zeros((6, 6))
    inplane = [a for a in range(3) if a != axis]
    for a in inplane:
        C[a, a] = fs * (P - lam * lam / P)
    a, b = inplane
    C[a, b] = C[b, a] = fs * (lam - lam * lam / P)
    C[{(0, 1): 5, (0, 2): 4, (1, 2): 3}[(a, b)], {(0, 1): 5, (0, 2): 4, (1, 2): 3}[(a, b)]] = fs * mu
    return C


@pytest.mark.parametrize("solver", SOLVERS)
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("mixed", 2e-5)])
def test_culled_laminate_and_limits_through_the_stiffness_entry(precision, tol, solver):
    # moduli given directly: zero culls a voxel.  Two free plates (closed form),
    # a fully solid cell (D), an empty cell (C = 0)
    A = api()
    n = 12
    prof = np.array([1, 1, 1, 0, 0, 1, 1, 1, 0, 0, 0, 0], dtype=np.float64)
    for axis in (0, 2):
        shape = [1, 1, 1]
        shape[2 - axis] = n
        E = torch.tensor(np.broadcast_to(prof.reshape(shape), (n, n, n)).copy(), device="cuda")
        r = A.homogenize_stiffness(E, 0.3, precision=precision, rtol=1e-10 if precision == "fp64" else 1e-6,
                                   solver=solver)
        ref = _plate(0.5, axis=axis)
        print("plates", axis, r["iters"], np.abs(r["C"] - ref).max(), flush=True)
        assert r["status"] == 0 and np.abs(r["C"] - ref).max() <= tol * np.abs(ref).max()
        assert r["active_nodes"] == 8 * n * n
    E = torch.full((n, n, n), 2.0, dtype=torch.float64, device="cuda")
    r = A.homogenize_stiffness(E, 0.3, precision=precision, solver=solver)
    lam, mu = 0.3 / (1.3 * 0.4), 1.0 / 2.6
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[np.arange(3), np.arange(3)] = lam + 2 * mu
    D[np.arange(3, 6), np.arange(3, 6)] = mu
    assert r["status"] == 0 and np.abs(r["C"] - 2.0 * D).max() <= 1e-12 * 2.0
    r = A.homogenize_stiffness(torch.zeros((n, n, n), dtype=torch.float64, device="cuda"), 0.3,
                               precision=precision, solver=solver)
    assert r["status"] == 0 and r["active_nodes"] == 0 and np.all(r["C"] == 0.0)


def test_multigrid_and_jacobi_preconditioners_agree_at_64():
    # the same culled system: the V-cycle changes the iteration count, not C^H
    A = api()
    d = wl.shell_128(2010, n=64)
    print("selective 64^3: multigrid vs Jacobi", flush=True)
    rm = A.homogenize(d, precision="mixed", rtol=3e-6, solver="selective")
    rj = A.homogenize(d, precision="mixed", rtol=3e-6, solver="selective-jacobi")
    print("  iters mg", rm["iters"].tolist(), "jacobi", rj["iters"].tolist(), flush=True)
    assert rm["status"] == 0 and rj["status"] == 0
    assert rm["active_nodes"] == rj["active_nodes"] and rm["V"] == rj["V"]
    assert_ch_close(rm["C"], rj["C"], 1e-4)
    assert 4 * max(rm["iters"]) < max(rj["iters"])


@pytest.mark.parametrize("solver", SOLVERS)
def test_batched_selective_solve_equals_single_designs(solver):
    # a batch shares every launch (grid y = design), each design keeps its own
    # reductions and schedule: results bit-identical to the designs alone
    A = api()
    designs = [wl.shell_128(2020, n=32), wl.shell_128(2021, n=40), wl.shell_128(2022, n=48)]
    print(f"{solver}: batch of {len(designs)} vs single", flush=True)
    rb = A.homogenize_batch(designs, precision="mixed", rtol=3e-6, solver=solver)
    for d, r in zip(designs, rb):
        r1 = A.homogenize(d, precision="mixed", rtol=3e-6, solver=solver)
        print("  n", d.n, "iters", r["iters"].tolist(), "active", r["active_nodes"], flush=True)
        assert r["status"] == 0 and r1["status"] == 0
        assert np.array_equal(r["C"], r1["C"]) and np.array_equal(r["iters"], r1["iters"])
        assert r["active_nodes"] == r1["active_nodes"]
