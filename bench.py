#!/usr/bin/env python3
"""Benchmark: homogenized designs/s at 128^3 through the served mixed-precision
path, with p50/p99 latency, the FP64 GPU path beside it, the C^H error of
mixed versus FP64, the HBM roofline fraction of the CG stencil kernel and the
FP64 CPU oracle timed on the host as a baseline.

One step = one batch of the 128^3 designs (48 charges, magnitudes U[-1,1]
shifted to zero net charge, volume fraction U[0.05, 0.15], void E = 1e-6)
submitted together to the continuous-batching engine and run to completion:
field -> threshold -> six-case PCG -> C^H for every design.

    python bench.py [--gpus 1] [--steps 2] [--warmup 1]

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Achievable read+write stream on this GPU: the library's plain 16-byte-vector
# copy kernel (shh_stream_copy) over 4 GiB, far above the 256 MB last-level
# cache, timed with HIP events by `bench.py --copy-only`
# (profiles/stream_copy_calibration.md).  Reported beside the 8 TB/s peak.
COPY_CEILING_GBS = 4912.5  # best of five 4 GiB copies (mean 4891.5)

# Measured memory traffic of the dominant kernel relative to its algorithmic
# bytes (rocprofv3 FETCH_SIZE x 2 and WRITE_SIZE x 1, the factors the 4 GiB
# stream copy gives; profiles/mg_apply_128_hbm_traffic.md), keyed by kernel
# family.  The counters count L2-to-fabric bytes, last-level-cache hits
# included, so the figure bounds HBM traffic from above.  It holds only for
# the kernel sources it was measured on (digest), null otherwise.
TRAFFIC = {
    "mg_apply1": {"ratio": 1.87, "sources": ["mg.hip", "mg.hpp", "common.hpp"],
                  "sha256": "722819f5a030965320042ddc7a7ee96a57fb468c25582d89fd867fff0140f3b0"},
}


def traffic_ratio(kind):
    import hashlib
    t = TRAFFIC.get(kind)
    if not t:
        return None
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2511_04025_amd", "csrc")
    for f in t["sources"]:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return t["ratio"] if h.hexdigest() == t["sha256"] else None


def family_bytes(results, n, R, solver, deg0=1):
    """Algorithmic HBM bytes per kernel family over the given results (FP32
    vectors, 12 B per node and load case per vector; a design's per-node data
    -- moduli, D^-1, coarse stencils -- counts once per iteration in which any
    of its load cases runs).  Only the work that each design's iteration
    counts imply is counted: restarted V-cycles after a residual replacement
    are not, so the figures are lower bounds.
      multigrid voxel level, per (node, load case), with the voxel level's
      Chebyshev degree deg0 (the library's build option; 1 by default):
        direction pass  48 (z, p read; p, q written) + 4 E per node
        pre-smoothing   48 (b staged; r, d1, x written) + 8 (E, D^-1) per node;
                        degree 1: 36 (b staged; r, x written) + 8
        r - K d1        36 (d1 staged, r read, r written) + 4 (degree 2 only)
        post-smoothing  36 (x staged, b read, r written) + 4 (degree 2 only)
        last sweep      48 (r staged; b, x read; x written) + 8; degree 1 the
                        one post-smoothing pass: 36 (x staged, b read, z
                        written) + 8
        CG update       72 (x, p, b, q read; x, b written)
        restriction     12 fine read + 12 per coarse node written
        prolongation    24 fine read and written + 12 per coarse node read
      first coarse level operator, 4 per iteration, each with the Chebyshev
        sweep after it in its output stage: 504 B of stencil per coarse node
        per pass + 36 B of D^-1 per coarse node, and per (coarse node, load
        case) 60 (d, b read; r, x, d1 written) + 36 (d1, r read; r written)
        + 60 (x, b read; r, d, x + d written) + 48 (d, x + d, r read; x written)
      FP64 residual: 24 (x64) + 12 (r) per (node, load case) + 8 (E) per node,
        every R iterations and once at the end
      Jacobi CG pass: 96 per (node, load case) + 8 per node
      selective solve, per (active node, running load case) and per active node:
        Jacobi-preconditioned:
        operator pass   36 (p, r read; q written) + 16 (coordinate, map entry,
                        modulus, D^-1)
        update          84 (x, p, r, q read; x, r, p written) + 4 (D^-1)
        multigrid-preconditioned, per iteration:
        q = K p         24 (p read, q written) + 12 (coordinate, map entry, modulus)
        smoothing       216 over the four fused operator passes (60 + 36 + 60 + 60)
                        + 64 (16 per pass); degree 1: 84 over two (48 + 36) + 32
        vectors         120 (CG update with D^-1 r: 84; p = z + beta p: 36) + 4
        transfers       36 per (active node, case) + 24 per (level-1 node, case)
                        + 4 per voxel (map) + 4 per active node (coordinate)
        FP64 residual   36 (x64 read, r written) + 20"""
    nn = n ** 3
    nn1 = nn // 8
    out = {k: 0.0 for k in ("cg_pass", "mg_dir", "mg_step1", "mg_res", "mg_post", "mg_last", "mg_update",
                            "mg_restrict", "mg_prolong", "mg_apply1", "resid64", "sel_op", "sel_update",
                            "sel_resid", "sel_mg_pq", "sel_mg_smooth", "sel_mg_vec", "sel_mg_transfer")}
    for r in results:
        it = [int(v) for v in r["iters"]]
        Ik, Im = sum(it), max(it)
        nres = [v // R + 1 for v in it]  # replacements, then the final check
        if solver in ("selective", "selective-jacobi"):
            na = float(r["active_nodes"])
            out["sel_resid"] += 36.0 * na * (sum(nres) + 6) + 20.0 * na * (max(nres) + 1)
            if solver == "selective-jacobi":
                out["sel_op"] += 36.0 * na * Ik + 16.0 * na * Im
                out["sel_update"] += 84.0 * na * Ik + 4.0 * na * Im
            else:
                out["sel_mg_pq"] += 24.0 * na * Ik + 12.0 * na * Im
                if deg0 == 1:
                    out["sel_mg_smooth"] += 84.0 * na * Ik + 32.0 * na * Im
                else:
                    out["sel_mg_smooth"] += 216.0 * na * Ik + 64.0 * na * Im
                out["sel_mg_vec"] += 120.0 * na * Ik + 4.0 * na * Im
                out["sel_mg_transfer"] += (36.0 * na + 24.0 * nn1) * Ik + (4.0 * nn + 4.0 * na) * Im
            continue
        out["resid64"] += 36.0 * nn * sum(nres) + 8.0 * nn * max(nres)
        if solver == "jacobi":
            out["cg_pass"] += 96.0 * nn * Ik + 8.0 * nn * Im
            continue
        out["mg_dir"] += 48.0 * nn * Ik + 4.0 * nn * Im
        if deg0 == 1:
            out["mg_step1"] += 36.0 * nn * Ik + 8.0 * nn * Im
            out["mg_last"] += 36.0 * nn * Ik + 8.0 * nn * Im
        else:
            out["mg_step1"] += 48.0 * nn * Ik + 8.0 * nn * Im
            out["mg_res"] += 36.0 * nn * Ik + 4.0 * nn * Im
            out["mg_post"] += 36.0 * nn * Ik + 4.0 * nn * Im
            out["mg_last"] += 48.0 * nn * Ik + 8.0 * nn * Im
        out["mg_update"] += 72.0 * nn * Ik
        out["mg_restrict"] += (12.0 * nn + 12.0 * nn1) * Ik
        out["mg_prolong"] += (24.0 * nn + 12.0 * nn1) * Ik
        out["mg_apply1"] += (4 * 504.0 + 36.0) * nn1 * Im + 204.0 * nn1 * Ik
    return out


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--designs", type=int, default=8)
    # CG tolerance of the served path, ||f - K u|| / ||f||: 3e-6 with either solver keeps
    # every C^H entry within 1e-4 of the oracle on the eight 48^3 designs (1e-5 misses it on
    # one of them: 1.27e-4 on an entry at 2e-3 of the largest) and of the FP64 path at 128^3.
    # The run checks it on the FP64 subset.
    ap.add_argument("--rtol", type=float, default=None,
                    help="CG tolerance (default 3e-6)")
    ap.add_argument("--solver", default="mg", choices=["mg", "jacobi", "selective", "selective-jacobi"],
                    help="CG preconditioner: geometric multigrid V-cycle or Jacobi; selective: the culled "
                         "solve on the active nodes, the designs of a step batched (multigrid-preconditioned, or "
                         "Jacobi-preconditioned with selective-jacobi)")
    ap.add_argument("--fp64-designs", type=int, default=8, help="designs also run on the FP64 GPU path")
    ap.add_argument("--jacobi-designs", type=int, default=8,
                    help="with --solver mg: designs also run with the Jacobi-preconditioned CG (mixed)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="budget of the oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--iters-per-step", type=int, default=4,
                    help="engine iterations between polls (admission and retirement happen at polls)")
    ap.add_argument("--recompute-every", type=int, default=0,
                    help="FP64 residual replacement period R (0: the library default, 50)")
    ap.add_argument("--max-iter", type=int, default=20000,
                    help="CG iteration cap (lower it only for hardware-counter runs)")
    ap.add_argument("--copy-only", action="store_true",
                    help="run a plain 1 GiB device-to-device copy (counter calibration) and exit")
    ap.add_argument("--mode", default="homogenize", choices=["homogenize", "serving-trace", "inverse-step"],
                    help="homogenize: the headline line; serving-trace: Poisson trace of mixed resolutions; "
                         "inverse-step: batched forward + adjoint of the bulk/Poisson loss")
    ap.add_argument("--trace-count", type=int, default=64, help="requests in the serving trace")
    ap.add_argument("--rate", type=float, default=0.0, help="arrival rate (requests/s); 0: 0.7 x saturated")
    ap.add_argument("--arena-gb", type=float, default=64.0, help="engine arena for the serving trace")
    ap.add_argument("--inverse-batch", type=int, default=32)
    ap.add_argument("--inverse-n", type=int, default=96)
    return ap.parse_args()


def serving_trace(args):
    """Poisson arrivals of requests with n in {64, 96, 128}, 16-64 charges and
    V in [0.03, 0.2] against the continuous-batching engine."""
    import numpy as np
    import torch
    from paper_2511_04025_amd import serving, workloads as wl
    designs = wl.serving_trace(count=args.trace_count)
    engine = serving.Engine(int(args.arena_gb * (1 << 30)), max_slots=256, precision="mixed", rtol=args.rtol,
                            solver=args.solver)
    rate = args.rate
    if rate <= 0:
        # saturated throughput of a closed batch of the first 16 requests
        t0 = time.perf_counter()
        for i, d in enumerate(designs[:16]):
            engine.submit(d, 10 ** 6 + i)
        got = 0
        while got < 16:
            engine.step(args.iters_per_step)
            got += len(engine.poll())
        sat = 16 / (time.perf_counter() - t0)
        rate = 0.7 * sat
        print(f"serving: saturated {sat:.3f} designs/s, arrival rate {rate:.3f}/s", file=sys.stderr, flush=True)
    arrivals = wl.poisson_arrivals(len(designs), rate)
    torch.cuda.synchronize()
    res, lat, wall = serving.run_trace(engine, designs, arrivals, iters_per_step=args.iters_per_step,
                                       timeout_s=3000.0)
    engine.close()
    L = np.array([lat[i] for i in range(len(designs))])
    bad = sum(1 for r in res.values() if r["status"] != 0)
    # the requests that did not converge: (index, n, status, worst relative residual)
    failed = [[int(i), int(designs[i].n), int(r["status"]), float(np.max(r["rel_res"]))]
              for i, r in sorted(res.items()) if r["status"] != 0]
    by_n = {}
    for i, d in enumerate(designs):
        by_n.setdefault(d.n, []).append(L[i])
    print(json.dumps({
        "metric": "serving trace: homogenized designs/s and latency (Poisson arrivals)",
        "value": round(len(designs) / wall, 4), "unit": "designs/s", "n_gpus": 1,
        "higher_is_better": True, "data": "synthetic",
        "config": {"workload": f"serving trace: {len(designs)} requests, n in {{64,96,128}}, N U{{16..64}}, "
                               f"V U[0.03,0.2], void E 1e-6, mixed, rtol {args.rtol}, solver {args.solver}",
                   "rate": round(rate, 4)},
        "latency_p50_s": round(float(np.percentile(L, 50)), 4),
        "latency_p99_s": round(float(np.percentile(L, 99)), 4),
        "latency_p50_by_n": {str(k): round(float(np.percentile(v, 50)), 4) for k, v in sorted(by_n.items())},
        "status_failures": bad, "failed_requests": failed, "wall_s": round(wall, 2)}))


def inverse_step(args):
    """One differentiable design step: forward of a batch at n^3 with the
    logistic shell (t fixed from V = 0.10 at the initial design), the
    bulk-modulus / Poisson-ratio loss, and the adjoint to charge positions and
    values through torch.autograd."""
    import numpy as np
    import torch
    from paper_2511_04025_amd import autograd as AG, workloads as wl
    designs = wl.smooth_shell_96_batch(n=args.inverse_n, count=args.inverse_batch)
    t = AG.initial_thickness(designs)
    spec = AG.Spec(n=args.inverse_n, thickness=t, kappa=designs[0].kappa, E_void=designs[0].E_void,
                   precision="mixed", rtol=args.rtol, solver=args.solver)
    pos = torch.tensor(np.stack([d.pos for d in designs]), dtype=torch.float64, requires_grad=True)
    q = torch.tensor(np.stack([d.q for d in designs]), dtype=torch.float64, requires_grad=True)
    times = []
    for step in range(args.warmup + args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        C, V = AG.Homogenize.apply(pos, q, spec)
        K_target = 0.5 * AG.voigt_bulk(C).detach().mean()
        L = AG.bulk_poisson_loss(C, K_target, 0.0)
        pos.grad = None
        q.grad = None
        L.backward()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        print(f"inverse: step {step} {dt:.2f} s loss {float(L.detach()):.4e}", file=sys.stderr, flush=True)
        if step >= args.warmup:
            times.append(dt)
    ms = 1e3 * float(np.mean(times))
    print(json.dumps({
        "metric": "differentiable design step: designs/s (forward + adjoint)",
        "value": round(args.inverse_batch / (ms / 1e3), 4), "unit": "designs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 1), "higher_is_better": True,
        "data": "synthetic",
        "config": {"workload": f"smooth_shell_96: batch {args.inverse_batch} at {args.inverse_n}^3, 32 charges +-1, "
                               f"logistic shell kappa=4n, t from V=0.10, mixed, rtol {args.rtol}, solver {args.solver}"},
        "grad_norm_pos": float(pos.grad.norm()), "grad_norm_q": float(q.grad.norm())}))


def copy_calibration():
    """The library's plain streaming copy at 4 GiB (far above the 256 MB
    last-level cache) and at 64 MiB (inside it), 5 times each, timed with HIP
    events on the stream it runs on.  Under rocprofv3 --pmc its FETCH_SIZE /
    WRITE_SIZE readings calibrate the HBM traffic counters."""
    import ctypes
    import torch
    from paper_2511_04025_amd import binding as B
    lib = B.lib()
    st = torch.cuda.current_stream()
    out = {}
    for nbytes in (4 << 30, 64 << 20):
        a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        ms = []
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            B.check(lib.shh_stream_copy(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()),
                                        ctypes.c_size_t(nbytes), ctypes.c_void_p(st.cuda_stream)), "shh_stream_copy")
            e1.record(st)
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        assert torch.equal(a, b)
        best = min(ms[1:])
        out[f"copy_{nbytes >> 20}MiB"] = {"bytes_each_way": nbytes, "ms": [round(v, 4) for v in ms],
                                          "rw_gbs_best": round(2 * nbytes / best / 1e6, 1),
                                          "rw_gbs_mean": round(2 * nbytes / (sum(ms[1:]) / 4) / 1e6, 1)}
        del a, b
        torch.cuda.empty_cache()
    print(json.dumps(out))


def cpu_baseline(design, gpu_iters, budget_s):
    """Time the oracle on a bounded sample and scale it to designs/s at n^3:
    field + assembly + a bounded number of CG iterations at 48^3 for the same
    design, extrapolated by n^3 and by the iteration count the oracle's solver
    (Jacobi-PCG) needs at n^3, as measured for the same algorithm on the GPU."""
    import numpy as np
    from oracle import fem, field as fld, solve as slv
    m = 48
    t0 = time.perf_counter()
    F, G = fld.field_and_gradient(design.pos, design.q, m)
    dist = fld.distance(F, G)
    t = fld.thickness_for_volume(dist, design.target_vf, 0.0)
    Ee = fld.stiffness_field(fld.occupancy(dist, t, 0.0), design.E, design.E_void)
    K = fem.assemble(Ee, design.nu, m)
    f = fem.load_vectors(Ee, design.nu, m)
    Kp, fp = slv.pin_node0(K, f)
    t_setup = time.perf_counter() - t0
    # CG iterations until the budget is used (the oracle's own loop, capped)
    left = max(budget_s - t_setup, 2.0)
    t1 = time.perf_counter()
    probe = 5
    slv.pcg_jacobi(Kp, fp, rtol=1e-300, maxiter=probe)
    t_probe = (time.perf_counter() - t1) / probe
    k = max(probe, min(400, int(left / max(t_probe, 1e-6))))
    t2 = time.perf_counter()
    slv.pcg_jacobi(Kp, fp, rtol=1e-300, maxiter=k)
    t_it = (time.perf_counter() - t2) / k
    scale = (design.n / m) ** 3
    est = t_setup * scale + gpu_iters * t_it * scale
    return {
        "value": 1.0 / est,
        "unit": "designs/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"oracle (NumPy/SciPy FP64) on the 48-charge shell design seed {design.seed} at {m}^3: field+threshold+"
                   f"assembly {t_setup:.2f} s, {k} Jacobi-PCG iterations {t_it * 1e3:.1f} ms each; scaled by "
                   f"({design.n}/{m})^3 and the {gpu_iters} Jacobi-PCG iterations one {design.n}^3 design needs; "
                   f"host os.cpu_count()={os.cpu_count()}, single-threaded SciPy/NumPy"),
    }


def main():
    args = parse()
    if args.rtol is None:
        args.rtol = 3e-6
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.copy_only:
        copy_calibration()
        return
    if args.mode == "serving-trace":
        serving_trace(args)
        return
    if args.mode == "inverse-step":
        inverse_step(args)
        return
    import numpy as np
    import torch

    from paper_2511_04025_amd import api, binding as B, serving, workloads as wl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    designs = wl.shell_128_designs(n=args.n, count=args.designs)
    eng_opts = dict(precision="mixed", rtol=args.rtol, max_iter=args.max_iter, solver=args.solver,
                    recompute_every=args.recompute_every)
    selective = args.solver in ("selective", "selective-jacobi")
    engine = None
    if not selective:
        probe = serving.Engine(1 << 20, max_slots=1, **eng_opts)
        fp = probe.footprint(designs[0])
        probe.close()
        del probe
        engine = serving.Engine(fp * args.designs + (64 << 20), max_slots=args.designs, **eng_opts)

    def one_step_selective():
        # the selective solve takes the step's designs in one batched call; a
        # design's latency runs from its own field stage to the batch's end
        t0 = time.perf_counter()
        res = api.homogenize_batch(designs, **eng_opts)
        lat = [r["ms"]["all"] / 1e3 for r in res]
        wall = time.perf_counter() - t0
        print(f"bench: selective step {wall:.2f} s, iters {[int(r['iters'].max()) for r in res]}", file=sys.stderr,
              flush=True)
        return res, lat

    def one_step():
        if selective:
            return one_step_selective()
        t0 = time.perf_counter()
        for i, d in enumerate(designs):
            engine.submit(d, i)
        res, lat = {}, {}
        while len(res) < len(designs):
            engine.step(args.iters_per_step)
            now = time.perf_counter() - t0
            for rid, r in engine.poll():
                res[rid] = r
                lat[rid] = now
                print(f"bench: design {rid} done at {now:.2f} s, iters {r['iters'].tolist()}, "
                      f"status {r['status']}", file=sys.stderr, flush=True)
        return [res[i] for i in range(len(designs))], [lat[i] for i in range(len(designs))]

    for _ in range(args.warmup):
        one_step()
    lib = B.lib()
    lib.shh_profile_enable(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    all_res, all_lat = [], []
    for _ in range(args.steps):
        res, lat = one_step()
        all_res += res
        all_lat += lat
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fam = {}
    for k, name in enumerate(B.PROF_KINDS):
        launches, ms = ctypes_int64(), ctypes_double()
        B.check(lib.shh_profile_read(k, launches, ms), "shh_profile_read")
        fam[name] = (launches.value, ms.value)
    lib.shh_profile_enable(0)
    ndes = args.steps * len(designs)
    value = ndes / wall
    ms_per_step = wall / args.steps * 1e3
    bad = [r["status"] for r in all_res if r["status"] != 0]

    # per-family roofline: algorithmic bytes implied by the iteration counts
    # over the event-timed milliseconds of that family's launches
    R = args.recompute_every if args.recompute_every > 0 else (10 if args.solver == "selective" else 50)
    # the voxel level's smoothing degree, from the passes that ran: degree 2
    # has the r - K d1 pass (dense) or two smoothing passes per transfer
    # (selective)
    if args.solver == "selective":
        deg0 = 2 if fam["sel_mg_smooth"][0] > fam["sel_mg_transfer"][0] else 1
    else:
        deg0 = 2 if fam["mg_res"][0] > 0 else 1
    fbytes = family_bytes(all_res, args.n, R, args.solver, deg0)
    kernels = {}
    for name, (nl, ms) in fam.items():
        if nl == 0:
            continue
        gbs = fbytes[name] / (ms / 1e3) / 1e9 if ms > 0 else 0.0
        kernels[name] = {"launches": nl, "ms": round(ms, 2), "avg_launch_ms": round(ms / nl, 4),
                         "algorithmic_bytes": int(fbytes[name]), "gbs": round(gbs, 1),
                         "frac": round(gbs / HBM_PEAK_GBS, 4)}
    dom = max(kernels, key=lambda k: kernels[k]["ms"])
    kd = kernels[dom]
    ratio = traffic_ratio(dom)
    per_launch = kd["algorithmic_bytes"] / kd["launches"]
    roofline = {
        "bound": "hbm", "achieved": kd["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": kd["frac"],
        "traffic": int(ratio * per_launch) if ratio is not None else None, "traffic_unit": "bytes/launch",
        "kernel": dom, "launches": kd["launches"], "avg_launch_ms": kd["avg_launch_ms"],
        "algorithmic_bytes_per_launch": int(per_launch),
        "copy_ceiling_gbs": COPY_CEILING_GBS,
    }
    tb = sum(v["algorithmic_bytes"] for v in kernels.values())
    tms = sum(v["ms"] for v in kernels.values())
    loop = {"algorithmic_bytes": int(tb), "timed_kernel_ms": round(tms, 1),
            "timed_kernels_gbs": round(tb / (tms / 1e3) / 1e9, 1) if tms > 0 else None,
            "timed_kernels_frac": round(tb / (tms / 1e3) / 1e9 / HBM_PEAK_GBS, 4) if tms > 0 else None,
            "wall_gbs": round(tb / wall / 1e9, 1), "wall_frac": round(tb / wall / 1e9 / HBM_PEAK_GBS, 4),
            "note": "bytes of every timed kernel family (lower bound: restarts not counted) over their "
                    "summed event time, and over the whole timed region's wall time"}

    # FP64 GPU path on a subset, and the C^H error of mixed vs FP64
    fp64 = {}
    if args.fp64_designs > 0:
        sub = designs[: args.fp64_designs]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        r64 = api.homogenize_batch(sub, precision="fp64", rtol=1e-10 if not selective else 1e-9,
                                   solver=args.solver)
        torch.cuda.synchronize()
        w64 = time.perf_counter() - t1
        errs, small = [], []
        for k, r in enumerate(r64):
            C, Cm = r["C"], all_res[k]["C"]
            s = np.abs(C).max()
            big = np.abs(C) >= 1e-3 * s
            errs.append(float(np.max(np.abs(Cm - C)[big] / np.abs(C)[big])))
            # entries below 1e-3 max|C|: absolute error relative to max|C| (bar 1e-7)
            small.append(float(np.max(np.abs(Cm - C)[~big], initial=0.0) / s))
        fp64 = {"fp64_designs_per_s": round(len(sub) / w64, 4), "ch_max_rel_err_vs_fp64": max(errs),
                "ch_small_entry_err_vs_fp64": max(small),
                "fp64_iters_mean": float(np.mean([r["iters"].max() for r in r64]))}

    # the Jacobi-preconditioned path on the same designs: the comparison, and
    # the iteration count of the oracle's own (Jacobi-PCG) solver
    jac = {}
    if args.solver == "mg" and args.jacobi_designs > 0:
        sub = designs[: args.jacobi_designs]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rj = api.homogenize_batch(sub, precision="mixed", rtol=args.rtol, max_iter=args.max_iter)
        torch.cuda.synchronize()
        wj = time.perf_counter() - t1
        jac = {"jacobi_designs_per_s": round(len(sub) / wj, 4),
               "jacobi_iters_mean": float(np.mean([r["iters"].max() for r in rj]))}

    iters = [int(r["iters"].max()) for r in all_res]
    out = {
        "metric": "homogenized designs/sec at 128^3 (C^H rel err <=1e-4 vs FP64) + p50/p99 latency",
        "value": round(value, 4),
        "unit": "designs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 stencil/vectors, f64 dots/recompute/reduction",
        "solver": args.solver,
        "data": "synthetic",
        "config": {"workload": f"shell_128: {len(designs)} designs/step at {args.n}^3, 48 charges, "
                               f"vf U[0.05,0.15], void E 1e-6, mixed precision, rtol {args.rtol}, "
                               + {"mg": "multigrid-preconditioned CG, continuous-batching engine",
                                  "jacobi": "Jacobi-preconditioned CG, continuous-batching engine",
                                  "selective": "selective (culled, beta > 1e-3) CG on the active nodes with "
                                               "the culled multigrid V-cycle, the step's designs batched in every launch",
                                  "selective-jacobi": "selective (culled, beta > 1e-3) Jacobi-PCG on the active "
                                                      "nodes, the step's designs batched in every launch"}[args.solver],
                   "n": args.n, "designs_per_step": len(designs)},
        "latency_p50_s": round(float(np.percentile(all_lat, 50)), 4),
        "latency_p99_s": round(float(np.percentile(all_lat, 99)), 4),
        "cg_iters_mean": float(np.mean(iters)),
        "active_node_fraction_mean": float(np.mean([r["active_nodes"] for r in all_res])) / args.n ** 3,
        "status_failures": len(bad),
        "roofline": roofline,
        "loop_roofline": loop,
        "kernels": kernels,
    }
    out.update(fp64)
    out.update(jac)
    if not args.no_cpu:
        oracle_iters = int(jac.get("jacobi_iters_mean", np.mean(iters))) if args.solver == "mg" else int(np.mean(iters))
        out["cpu_baseline"] = cpu_baseline(designs[0], oracle_iters, args.cpu_seconds)
    if engine is not None:
        engine.close()
    print(json.dumps(out))


def ctypes_int64():
    import ctypes
    return ctypes.c_int64(0)


def ctypes_double():
    import ctypes
    return ctypes.c_double(0.0)


if __name__ == "__main__":
    main()
