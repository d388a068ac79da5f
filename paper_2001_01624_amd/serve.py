"""Continuous-batching request loop over the C-ABI solver.

Requests (a model plus one or more source vectors) arrive over time.  The
dispatcher admits the oldest waiting request as soon as a slot is idle and
its device footprint fits the free part of the HBM budget; admitted requests
run concurrently, each on its own HIP stream in its own worker thread (the C
calls release the GIL), so their kernels overlap on the device.  A request
keeps its context (operator, bases, coarse inverses) resident for all of its
solves; from the second solve on, the increments between consecutive
solutions become dynamic stages (newest first, at most two).  Every solve
runs to the requested relative residual on the FP64 residual.

Each request owns an independent context and every reduction in the library
has a fixed order, so a request's results do not depend on what else runs.
"""
from __future__ import annotations

import queue
import threading
import time

import numpy as np

from . import capi


def request_footprint(req, options) -> int:
    """Device bytes a request may hold: the context, its vectors and two
    dynamic stages (coarse matrices sized by the dynamic-block cap)."""
    N = int(np.prod(req.problem.dims))
    base = capi.footprint_bytes(req.problem, req.partitions, options)
    if base == 0:
        return 0
    mdyn = min(options.max_dyn_blocks, int(req.problem.n_active))
    mp = -(-mdyn // 64) * 64  # coarse matrices are padded to the 64-wide inverse tiles
    # per stage: block map and cell list, A_c and its inverse, coarse vectors;
    # plus a coarse-inverse panel of that height should it outgrow the set-up one
    dyn = 2 * (8 * N + 16 * mp * mp + 24 * mp) + 8 * (mp + 128) * 64
    vecs = 8 * N * (4 + len(req.sources))
    return int(base + dyn + vecs)


class Server:
    def __init__(self, slots=8, hbm_budget=64 << 30, options=None, rtol=1e-6, max_iters=3000, max_sweeps=100,
                 basis_tol=1e-3, keep_solutions=False, dynamic=True):
        import torch

        self.torch = torch
        self.slots = slots
        self.budget = int(hbm_budget)
        self.options = options if options is not None else capi.default_options(smoother="ilu0_line", outer="gmres")
        self.rtol, self.max_iters = rtol, max_iters
        self.max_sweeps, self.basis_tol = max_sweeps, basis_tol
        self.keep = keep_solutions
        self.dynamic = dynamic
        self.streams = [torch.cuda.Stream() for _ in range(slots)]

    # -- one request on one slot ---------------------------------------------
    def _run(self, req, stream):
        torch = self.torch
        with torch.cuda.stream(stream):
            g = capi.Solver(req.problem, req.partitions, self.options, stream=stream)
            try:
                for k in range(len(req.partitions)):
                    g.update_basis(stage=k, max_sweeps=self.max_sweeps, tol=self.basis_tol)
                N = g.N
                x = torch.zeros(N, dtype=torch.float64, device="cuda")
                prev = []
                for q in req.sources:
                    qd = torch.as_tensor(q).to("cuda", non_blocking=False)
                    if self.dynamic and len(prev) >= 2:
                        incs = [prev[-1] - prev[-2]] + ([prev[-2] - prev[-3]] if len(prev) >= 3 else [])
                        req.dyn_blocks.append(g.add_dynamic_basis(incs))
                    it, rel, rc = g.solve(x, source=qd, rtol=self.rtol, max_iters=self.max_iters)
                    req.iters.append(it)
                    req.relres.append(rel)
                    req.status.append(rc)
                    prev.append(x.clone())
                    if len(prev) > 3:
                        prev.pop(0)
                    if self.keep:
                        req.solutions.append(x.cpu().numpy().copy())
                stream.synchronize()
            finally:
                g.close()

    # -- the loop ------------------------------------------------------------
    def run(self, requests, realtime=True):
        """Serve `requests` (arrival times in seconds from start).  Returns a
        dict of aggregate statistics; per-request results are stored on the
        request objects."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        foot = {r.rid: request_footprint(r, self.options) for r in reqs}
        for r in reqs:
            if foot[r.rid] == 0 or foot[r.rid] > self.budget:
                r.error = "request does not fit the HBM budget" if foot[r.rid] else "invalid request"
        todo = [r for r in reqs if not r.error]
        lock = threading.Condition()
        state = {"free": self.budget, "idle": list(range(self.slots)), "running": 0}
        done_q = queue.Queue()

        def worker(req, slot):
            try:
                self._run(req, self.streams[slot])
            except Exception as exc:  # reported per request, the loop continues
                req.error = f"{type(exc).__name__}: {exc}"
            req.finished = time.perf_counter() - t0
            with lock:
                state["free"] += foot[req.rid]
                state["idle"].append(slot)
                state["running"] -= 1
                lock.notify_all()
            done_q.put(req.rid)

        t0 = time.perf_counter()
        waiting = []
        nxt = 0
        threads = []
        with lock:
            while True:
                now = time.perf_counter() - t0
                while nxt < len(todo) and (not realtime or todo[nxt].arrival <= now):
                    waiting.append(todo[nxt])
                    nxt += 1
                # admit the oldest waiting request while a slot is idle and it fits
                while waiting and state["idle"] and foot[waiting[0].rid] <= state["free"]:
                    r = waiting.pop(0)
                    slot = state["idle"].pop(0)
                    state["free"] -= foot[r.rid]
                    state["running"] += 1
                    r.admitted = time.perf_counter() - t0
                    th = threading.Thread(target=worker, args=(r, slot), daemon=True)
                    threads.append(th)
                    th.start()
                if nxt >= len(todo) and not waiting and state["running"] == 0:
                    break
                timeout = None
                if nxt < len(todo):
                    timeout = max(0.0, todo[nxt].arrival - (time.perf_counter() - t0))
                lock.wait(timeout=timeout)
        for th in threads:
            th.join()
        makespan = time.perf_counter() - t0
        ok = [r for r in todo if not r.error]
        lat = np.array([r.finished - r.arrival for r in ok]) if ok else np.zeros(1)
        cells = sum(r.cells for r in ok)
        return {
            "requests": len(reqs),
            "completed": len(ok),
            "rejected": sum(1 for r in reqs if r.error),
            "solves": sum(len(r.sources) for r in ok),
            "cells": cells,
            "makespan_s": makespan,
            "cells_per_s": cells / makespan if makespan > 0 else 0.0,
            "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "all_converged": all(all(s == 0 for s in r.status) for r in ok),
            "max_relres": max((max(r.relres) for r in ok if r.relres), default=0.0),
        }


def run_ensemble(requests, options=None, chunk=64, threads=8, rtol=1e-6, max_iters=3000, max_sweeps=100,
                 basis_tol=1e-3, keep_solutions=False):
    """Solve an ensemble available at once (one stage and one source per
    request) in batches of ``chunk`` members (``msrsb_batch_*``: one launch
    per kernel over a batch), pipelined: ``threads - 1`` host threads set up
    the next batch's contexts and tear down the previous one's while the
    current batch runs on the device.  Each member's results are those of
    solving it alone, bit for bit.  Returns aggregate statistics; per-request
    results are stored on the request objects."""
    from concurrent.futures import ThreadPoolExecutor

    import torch

    opts = options if options is not None else capi.default_options(smoother="ilu0_line", outer="gmres")
    reqs = list(requests)
    groups = [reqs[k:k + chunk] for k in range(0, len(reqs), chunk)]
    # each set-up thread enqueues on a stream of its own, each batch runs on
    # its own stream: set-up, device work and teardown never wait for each
    # other's queued work
    local = threading.local()
    t0 = time.perf_counter()

    def setup(r):
        if not hasattr(local, "stream"):
            local.stream = torch.cuda.Stream()
        return capi.Solver(r.problem, r.partitions, opts, stream=local.stream)

    def teardown(gs, xs, rs):
        for g, x, r in zip(gs, xs, rs):
            if keep_solutions:
                r.solutions.append(x.cpu().numpy())
            g.close()
            r.finished = time.perf_counter() - t0

    with ThreadPoolExecutor(max(1, threads - 1)) as ex:
        pending = [ex.submit(setup, r) for r in groups[0]] if groups else []
        tails = []
        for k, grp in enumerate(groups):
            gs = [f.result() for f in pending]
            pending = [ex.submit(setup, r) for r in groups[k + 1]] if k + 1 < len(groups) else []
            stream = torch.cuda.Stream()
            with torch.cuda.stream(stream):
                xs = [torch.zeros(g.N, dtype=torch.float64, device="cuda") for g in gs]
                qs = [torch.as_tensor(np.asarray(r.sources[0], dtype=np.float64)).to("cuda", non_blocking=False)
                      for r in grp]
            b = capi.Batch(gs, stream=stream)
            try:
                b.update_basis(max_sweeps=max_sweeps, tol=basis_tol)
                it, rel, st = b.solve(xs, sources=qs, rtol=rtol, max_iters=max_iters)
            finally:
                b.close()
            for r, i, e, s in zip(grp, it, rel, st):
                r.iters.append(i)
                r.relres.append(e)
                r.status.append(s)
            tails.append(ex.submit(teardown, gs, xs, grp))
        for f in tails:
            f.result()
    makespan = time.perf_counter() - t0
    cells = sum(r.cells for r in reqs)
    return {
        "requests": len(reqs),
        "completed": len(reqs),
        "solves": len(reqs),
        "cells": cells,
        "makespan_s": makespan,
        "cells_per_s": cells / makespan if makespan > 0 else 0.0,
        "all_converged": all(all(s == 0 for s in r.status) for r in reqs),
        "max_relres": max((max(r.relres) for r in reqs if r.relres), default=0.0),
    }
