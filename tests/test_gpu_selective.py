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


def _sweep_design(index):
    # design `index` of a seeded random sweep (16 ... 128^3, 8-64 charges,
    # 3-30 % volume, nu from -0.3 to 0.45)
    rng = np.random.default_rng(777)
    for i in range(index + 1):
        n = int(rng.choice([32, 48, 64, 80, 96, 128]))
        d = wl.random_design(50000 + i, n, N=int(rng.integers(8, 64)), vf=float(rng.uniform(0.03, 0.3)),
                             E_void=float(rng.choice([1e-6, 1e-4, 1e-3])), pm=bool(rng.random() < 0.5))
        d = d.with_(nu=float(rng.choice([0.0, 0.2, 0.3, 0.45, -0.3])))
    return d


@pytest.mark.parametrize("index", [18, 34])
def test_designs_whose_kept_direction_lost_definiteness_converge(index):
    # on these two designs a CG direction kept across a residual replacement
    # once made p.Kp or r.z non-positive (a breakdown); the stalled load case
    # now resumes from a restart and the solve converges to the FP64 result
    A = api()
    d = _sweep_design(index)
    print(f"sweep design {index}: n {d.n}", flush=True)
    r = A.homogenize(d, precision="mixed", rtol=3e-6, solver="selective")
    print("  iters", r["iters"].tolist(), "status", r["status"], flush=True)
    assert r["status"] == 0 and np.all(r["rel_res"] <= 3e-6)
    r64 = A.homogenize(d, precision="fp64", rtol=1e-10, solver="selective")
    assert r64["status"] == 0
    assert_ch_close(r["C"], r64["C"], 1e-4)


def test_serving_trace_designs_at_the_fp32_limit():
    # two 64^3 requests of the 512-request serving trace.  Design 333 (12.6 %
    # volume): its mixed culled solve needs 1,100-3,800 iterations (FP64:
    # 145) and with degree-2 voxel smoothing reaches the tolerance and the
    # FP64 result; with degree 1 two load cases stalled above it.
    # Design 184 (3.5 % volume) sits below what FP32 vectors resolve on its
    # culled system: the mixed solve stops NOT_CONVERGED near 2e-5 (the
    # stagnation stop) instead of drifting, and FP64 converges.
    A = api()
    trace = wl.serving_trace(count=512)
    d = trace[333]
    r = A.homogenize(d, precision="mixed", rtol=3e-6, solver="selective")
    print("design 333: iters", r["iters"].tolist(), "status", r["status"], flush=True)
    assert r["status"] == 0 and np.all(r["rel_res"] <= 3e-6)
    r64 = A.homogenize(d, precision="fp64", rtol=1e-10, solver="selective")
    assert r64["status"] == 0
    # entries above 1e-3 of max|C| within 1e-4; the small ones carry 1.7e-7
    # of max|C| (the usual bar is 1e-7): FP32 on a poorly conditioned system
    assert_ch_close(r["C"], r64["C"], 1e-4, abs_tol=1e-6)
    d = trace[184]
    r = A.homogenize(d, precision="mixed", rtol=3e-6, solver="selective")
    print("design 184: iters", r["iters"].tolist(), "status", r["status"],
          [f"{v:.1e}" for v in r["rel_res"]], flush=True)
    assert r["status"] in (0, 1) and np.all(r["rel_res"] <= 1e-4)
    r64 = A.homogenize(d, precision="fp64", rtol=1e-10, solver="selective")
    assert r64["status"] == 0 and np.all(r64["rel_res"] <= 1e-10)


@pytest.mark.parametrize("precision,rtol,tol", [("fp64", 1e-12, 1e-8), ("mixed", 1e-7, 1e-4)])
def test_culled_gradient_matches_the_oracle(precision, rtol, tol):
    # the adjoint of Eq. (9) through the culled system (dE_e/dbeta_e = E on
    # active voxels, nothing on culled ones) against the oracle's
    A = api()
    from oracle import field as fld, selective as osel
    n = 12
    d = wl.random_design(63, n, N=6, vf=0.25, E_void=1e-3, kappa=4.0 * n)
    F, G = fld.field_and_gradient(d.pos, d.q, n)
    t = fld.thickness_for_volume(fld.distance(F, G), 0.25, d.kappa)
    rng = np.random.default_rng(9)
    dLdC = rng.standard_normal((6, 6))
    C_o, V_o, dpos_o, dq_o = osel.design_gradient_selective(d.pos, d.q, n, dLdC, 0.2, thickness=t, kappa=d.kappa)
    dt = d.with_(thickness=t)
    r = A.homogenize(dt, precision=precision, rtol=rtol, save_for_backward=True, return_workspace=True,
                     solver="selective")
    assert r["status"] == 0 and abs(r["V"] - V_o) <= 1e-13
    dpos, dq = A.grad(dt, r["opts"], r["workspace"], dLdC, 0.2)
    scale = max(np.abs(dpos_o).max(), np.abs(dq_o).max())
    print(f"culled gradient {precision}: pos {np.abs(dpos - dpos_o).max() / scale:.2e} "
          f"q {np.abs(dq - dq_o).max() / scale:.2e}", flush=True)
    assert np.max(np.abs(dpos - dpos_o)) <= tol * scale
    assert np.max(np.abs(dq - dq_o)) <= tol * scale


def test_culled_gradient_in_alpha_and_t_matches_differences():
    # alpha_hkl and t through the culled system, against central differences
    # of the GPU forward in FP64 (h small enough that no voxel crosses eps)
    A = api()
    n = 16
    d = wl.random_design(64, n, N=8, vf=0.2, E_void=1e-3, kappa=4.0 * n)
    alpha = 1.0 + 0.2 * np.random.default_rng(64).standard_normal((4, 4, 4))
    r0 = A.homogenize(d.with_(alpha=alpha), precision="fp64", rtol=1e-13, solver="selective")
    dd = d.with_(alpha=alpha, thickness=r0["t"], target_vf=None)
    w = np.random.default_rng(65).standard_normal((6, 6))
    r = A.homogenize(dd, precision="fp64", rtol=1e-13, save_for_backward=True, return_workspace=True,
                     solver="selective")
    gp, gq, ga, gt = A.grad(dd, r["opts"], r["workspace"], w, 0.3, full=True)
    ga = np.asarray(ga).reshape(alpha.shape)

    def loss(design):
        rr = A.homogenize(design, precision="fp64", rtol=1e-13, solver="selective")
        return float(np.sum(w * rr["C"]) + 0.3 * rr["V"])

    h = 1e-6
    for idx in ((0, 0, 0), (1, 2, 3)):
        ap, am = alpha.copy(), alpha.copy()
        ap[idx] += h
        am[idx] -= h
        fd = (loss(dd.with_(alpha=ap)) - loss(dd.with_(alpha=am))) / (2 * h)
        print("alpha", idx, fd, ga[idx], flush=True)
        assert abs(fd - ga[idx]) <= 2e-5 * np.abs(ga).max()
    fd = (loss(dd.with_(thickness=r0["t"] + h)) - loss(dd.with_(thickness=r0["t"] - h))) / (2 * h)
    print("t", fd, gt, flush=True)
    assert abs(fd - gt) <= 2e-5 * abs(gt)


def _drain(eng, got, iters):
    nr, nq = eng.step(iters)
    for rid, r in eng.poll():
        got[rid] = r
    return nr, nq


def test_engine_serves_the_selective_solve():
    # the continuous-batching engine with the selective solver: four 48^3
    # designs arriving in two waves between steps of uneven length; every
    # result is bit-for-bit the one the design gets alone and within the
    # per-entry bar of the culled oracle's stored values
    from paper_2511_04025_amd import serving
    seeds = (2000, 2001, 2002, 2003)
    designs = [wl.shell_128(s, n=48) for s in seeds]
    kw = dict(precision="mixed", rtol=3e-6, solver="selective")
    alone = {}
    for i, d in enumerate(designs):
        eng = serving.Engine(1 << 30, max_slots=2, **kw)
        eng.submit(d, i)
        got = {}
        for _ in range(400):
            nr, nq = _drain(eng, got, 16)
            if nr == 0 and nq == 0:
                break
        eng.close()
        alone[i] = got[i]
    print("selective engine: staggered mix", flush=True)
    eng = serving.Engine(1 << 30, max_slots=4, **kw)
    got = {}
    waves = {0: [0, 1], 2: [2, 3]}
    steps = [5, 3, 7, 4]
    for k in range(2000):
        for i in waves.get(k, []):
            eng.submit(designs[i], i)
        nr, nq = _drain(eng, got, steps[k % len(steps)])
        if k > 2 and nr == 0 and nq == 0:
            break
    eng.close()
    assert sorted(got) == list(range(4))
    for i, s in enumerate(seeds):
        r = got[i]
        g = golden(f"selective_n48_seed{s}.json")
        print(f"  seed {s}: iters {r['iters'].tolist()} alone {alone[i]['iters'].tolist()}", flush=True)
        assert r["status"] == 0 and r["active_nodes"] == g["active_nodes"]
        assert np.array_equal(r["C"], alone[i]["C"]) and np.array_equal(r["iters"], alone[i]["iters"])
        assert_ch_close(r["C"], np.array(g["C"]), 1e-4)
