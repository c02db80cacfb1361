"""Write the stored expected values under tests/golden/ by running the FP64
oracle (and nothing else) on the seeded workloads.

    python tests/golden/make_golden.py [small] [shell48] [smooth] [sel] [--procs 8]

small: 24^3, 16 charges of +-1, V = 0.12, void E 1e-3              -> small_shell_n24_seed1.json
shell48: 48^3 versions of the 128^3 designs (seeds 2000-2007), void 1e-6 -> shell_n48_seed<s>.json
smooth: 24^3 logistic designs (seeds 5000, 5001), kappa = 4n, t from V = 0.10,
    void 1e-6, with the oracle's design gradients of two functionals of
    (C^H, V): the bulk/Poisson loss, and a fixed random linear functional
    -> smooth_shell_n24_seed<s>.json
sel: the selective (culled, Sec. 4.2) oracle on the 48^3 designs (seeds
    2000-2003), on the 24^3 design of `small`, and on the 24^3 logistic design
    5000 (voxels with beta <= 1e-3 culled) -> selective_n<n>_seed<s>.json
All dense solves: Jacobi-PCG to ||r|| <= 1e-12 ||f|| (node 0 pinned); the
selective ones: Jacobi-PCG on the active nodes to the same tolerance.
"""
import json
import os
import sys
import time
from multiprocessing import Pool

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import adjoint as adj, fem, field as fld, homogenize as hom, metrics  # noqa: E402
from oracle import selective as sel  # noqa: E402
from paper_2511_04025_amd import workloads as wl  # noqa: E402


def _dump(path, obj):
    with open(path, "w") as f:
        json.dump(obj, f, indent=1)


def run_small(_=None):
    d = wl.small_shell_24()
    t0 = time.time()
    C, info = hom.homogenize_design(d.pos, d.q, d.n, target_vf=d.target_vf, E_void=d.E_void, rtol=1e-12)
    _dump(os.path.join(HERE, "small_shell_n24_seed1.json"), {
        "source": "oracle, make_golden.py small", "seed": 1, "n": 24, "C": C.tolist(), "V": info["V"],
        "t": info["t"], "iters": info["iters"].tolist(), "rel_res": info["rel_res"].tolist(),
        "seconds": time.time() - t0})
    return "small"


def run_shell48(seed):
    d = wl.shell_128(seed, n=48)
    t0 = time.time()
    C, info = hom.homogenize_design(d.pos, d.q, 48, target_vf=d.target_vf, E_void=d.E_void, rtol=1e-12,
                                    maxiter=400000)
    _dump(os.path.join(HERE, f"shell_n48_seed{seed}.json"), {
        "source": "oracle, make_golden.py shell48", "seed": seed, "n": 48, "target_vf": d.target_vf,
        "C": C.tolist(), "V": info["V"], "t": info["t"], "iters": info["iters"].tolist(),
        "rel_res": info["rel_res"].tolist(), "seconds": time.time() - t0})
    return f"shell48 {seed}"


def smooth_functionals(C, V):
    """The bulk/Poisson loss with targets fixed from the design itself (half the
    Hashin-Shtrikman bulk bound at its V, Poisson ratio 0), and a fixed random
    symmetric linear functional with dL/dV = 0.7."""
    lam, mu = fem.lame(1.0, 0.3)
    K1 = lam + 2.0 * mu / 3.0
    lv, mv = fem.lame(1e-6, 0.3)
    KU, _ = metrics.hashin_shtrikman_upper(V, K1, mu, lv + 2.0 * mv / 3.0, mv)
    K_target = 0.5 * KU
    g_loss = adj.bulk_poisson_loss_grad(C, K_target, 0.0)
    rng = np.random.default_rng(77)
    G = rng.standard_normal((6, 6))
    return K_target, g_loss, 0.5 * (G + G.T)


def run_smooth(seed):
    d = wl.smooth_shell_96(seed, n=24)
    t0 = time.time()
    F, G = fld.field_and_gradient(d.pos, d.q, 24)
    t = fld.thickness_for_volume(fld.distance(F, G), 0.10, d.kappa)
    C, info = hom.homogenize_design(d.pos, d.q, 24, thickness=t, kappa=d.kappa, E_void=d.E_void, rtol=1e-12,
                                    maxiter=400000)
    K_target, g_loss, g_rand = smooth_functionals(C, info["V"])
    gp_l, gq_l = adj.design_gradient(info, d.pos, d.q, 24, g_loss, 0.0, kappa=d.kappa, E_void=d.E_void)
    gp_r, gq_r = adj.design_gradient(info, d.pos, d.q, 24, g_rand, 0.7, kappa=d.kappa, E_void=d.E_void)
    _dump(os.path.join(HERE, f"smooth_shell_n24_seed{seed}.json"), {
        "source": "oracle, make_golden.py smooth", "seed": seed, "n": 24, "kappa": d.kappa, "t": t,
        "C": C.tolist(), "V": info["V"], "iters": info["iters"].tolist(), "rel_res": info["rel_res"].tolist(),
        "K_target": K_target, "nu_target": 0.0,
        "loss": float(metrics.bulk_poisson_loss(C, K_target, 0.0)),
        "dL_dC_loss": g_loss.tolist(), "dpos_loss": gp_l.tolist(), "dq_loss": gq_l.tolist(),
        "dL_dC_rand": g_rand.tolist(), "dL_dV_rand": 0.7, "dpos_rand": gp_r.tolist(), "dq_rand": gq_r.tolist(),
        "seconds": time.time() - t0})
    return f"smooth {seed}"


def run_sel(key):
    if key == "small":
        d = wl.small_shell_24()
        kw = dict(target_vf=d.target_vf)
    elif key == "smooth":
        d = wl.smooth_shell_96(5000, n=24)
        F, G = fld.field_and_gradient(d.pos, d.q, 24)
        kw = dict(thickness=fld.thickness_for_volume(fld.distance(F, G), 0.10, d.kappa), kappa=d.kappa)
    else:
        d = wl.shell_128(int(key), n=48)
        kw = dict(target_vf=d.target_vf)
    t0 = time.time()
    C, info = sel.homogenize_design_selective(d.pos, d.q, d.n, rtol=1e-12, maxiter=400000, **kw)
    _dump(os.path.join(HERE, f"selective_n{d.n}_seed{d.seed}.json"), {
        "source": "oracle.selective, make_golden.py sel", "seed": d.seed, "n": d.n, "C": C.tolist(),
        "V": info["V"], "t": info["t"], "kappa": d.kappa, "iters": info["iters"].tolist(),
        "rel_res": info["rel_res"].tolist(), "active_voxels": info["n_active_voxels"],
        "active_nodes": info["n_active_nodes"], "seconds": time.time() - t0})
    return f"sel {key}"


def main():
    args = sys.argv[1:]
    procs = 8
    if "--procs" in args:
        procs = int(args[args.index("--procs") + 1])
    which = [a for a in args if a in ("small", "shell48", "smooth", "sel")] or ["small", "shell48", "smooth", "sel"]
    jobs = []
    if "small" in which:
        jobs.append((run_small, 0))
    if "smooth" in which:
        jobs += [(run_smooth, s) for s in (5000, 5001)]
    if "shell48" in which:
        jobs += [(run_shell48, 2000 + i) for i in range(8)]
    if "sel" in which:
        jobs += [(run_sel, k) for k in ("small", "smooth", "2000", "2001", "2002", "2003")]
    with Pool(procs) as pool:
        rs = [pool.apply_async(f, (a,)) for f, a in jobs]
        for r in rs:
            print(r.get(), flush=True)


if __name__ == "__main__":
    main()
