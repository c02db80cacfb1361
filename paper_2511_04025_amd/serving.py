"""Continuous-batching homogenization service over the libshellhom engine.

The engine (C++, shh_engine_*) keeps every admitted design resident in one
device arena -- its grids, CG vectors and device-side solver state -- and runs
each CG phase as one launch over all resident designs.  Requests are admitted
at iteration boundaries while a slot and arena memory are free (first fit),
and retire when their six load cases have converged.

``Engine`` wraps the C handle; ``run_trace`` replays a timed arrival trace
(Poisson arrivals) against it and reports per-request latency.
"""
import ctypes
import time
from ctypes import byref, c_int32, c_size_t, c_uint64, c_void_p

import numpy as np
import torch

from . import binding as B


class Engine:
    def __init__(self, arena_bytes, max_slots=64, precision="mixed", rtol=None, max_iter=20000,
                 recompute_every=0, check_every=0, solver="jacobi"):
        if not torch.cuda.is_available():
            raise RuntimeError("the engine needs a HIP GPU")
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device="cuda")
        self.opts = B.make_opts(precision, rtol, max_iter, recompute_every, False, check_every, solver)
        self.stream = torch.cuda.current_stream()
        h = c_void_p()
        B.check(B.lib().shh_engine_create(c_void_p(self.arena.data_ptr()), c_size_t(self.arena.numel()),
                                          int(max_slots), c_void_p(self.stream.cuda_stream), byref(h)),
                "shh_engine_create")
        self.h = h
        self._keep = {}

    def footprint(self, design):
        a = B.DesignArgs(design)
        nb = c_size_t(0)
        B.check(B.lib().shh_engine_footprint(byref(a.c), byref(self.opts), byref(nb)), "shh_engine_footprint")
        return nb.value

    def submit(self, design, request_id, opts=None):
        """Queue a request; `opts` (a binding.ShhOpts) overrides the engine's
        options for this request (same precision required)."""
        a = B.DesignArgs(design)
        o = self.opts if opts is None else opts
        rc = B.lib().shh_engine_submit(self.h, byref(a.c), byref(o), c_uint64(int(request_id)))
        B.check(rc, "shh_engine_submit")

    def step(self, iters=16):
        nr, nq = c_int32(0), c_int32(0)
        B.check(B.lib().shh_engine_step(self.h, int(iters), byref(nr), byref(nq)), "shh_engine_step")
        return nr.value, nq.value

    def poll(self, max_results=256):
        out = (B.ShhResult * max_results)()
        ids = (c_uint64 * max_results)()
        n = c_int32(0)
        B.check(B.lib().shh_engine_poll(self.h, out, ids, int(max_results), byref(n)), "shh_engine_poll")
        return [(int(ids[i]), B.result_dict(out[i])) for i in range(n.value)]

    def cancel(self, request_id):
        return B.lib().shh_engine_cancel(self.h, c_uint64(int(request_id)))

    def close(self):
        if self.h:
            B.lib().shh_engine_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_trace(engine, designs, arrivals, iters_per_step=16, timeout_s=600.0):
    """Replay requests `designs[i]` arriving at `arrivals[i]` seconds (sorted).
    Returns (results by id, latency_s by id, wall seconds)."""
    t0 = time.perf_counter()
    submitted = 0
    results, latency = {}, {}
    order = np.argsort(arrivals, kind="stable")
    total = len(designs)
    while len(results) < total:
        now = time.perf_counter() - t0
        while submitted < total and arrivals[order[submitted]] <= now:
            i = int(order[submitted])
            engine.submit(designs[i], i)
            submitted += 1
        resident, queued = engine.step(iters_per_step)
        done_t = time.perf_counter() - t0
        for rid, res in engine.poll():
            results[rid] = res
            latency[rid] = done_t - arrivals[rid]
        if resident == 0 and queued == 0 and submitted < total:
            # idle: wait for the next arrival
            nxt = arrivals[order[submitted]]
            dt = nxt - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(min(dt, 0.05))
        if time.perf_counter() - t0 > timeout_s:
            raise TimeoutError("trace did not finish")
    return results, latency, time.perf_counter() - t0
