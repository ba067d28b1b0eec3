"""Served eigensolve stream on one GPU: admission by device-memory footprint and
continuous batching.

Requests (cells of different size, cutoff, band count, k-point and precision)
arrive over time.  Each is admitted, oldest first, as soon as an execution
slot is free and its device footprint fits the memory budget; it then runs on
its own context and stream from its own host thread, so solves that arrive
while others are on the GPU overlap with them.  Blocks stay resident on the
device for the whole solve; only eigenvalues return to the host.

    python -m paper_0707_3405_amd.serve --requests 16 --rate 2.0

This module is orchestration only: every step of every solve runs in the
library's kernels through the C ABI.
"""
from __future__ import annotations

import argparse
import collections
import json
import sys
import threading
import time

import numpy as np

from ._binding import Context, PW_PREC_FP64, PW_PREC_MIXED, PW_ERR_NOT_CONVERGED


def footprint(w, prec):
    """(npw, bytes): device memory one solve of workload w needs, sized on a
    host-only context (no GPU call)."""
    hc = Context(-1)
    npw = hc.init_basis(w.cell, w.kfrac, w.ecut, (w.n,) * 3)
    ws = hc.workspace_size(w.nbands, w.block, prec)
    hc.close()
    ldp = (npw + 31) // 32 * 32
    n3 = w.n ** 3
    proj = ldp * w.nproj * (16 + (8 if prec != PW_PREC_FP64 else 0))
    pot = n3 * 8 * 2 + (n3 * 4 if prec != PW_PREC_FP64 else 0)   # V, its staging copy, float copy
    tables = npw * (8 + 4 + 24) + 4096 * 8
    vectors = npw * w.nbands * 16                                    # the caller's X
    return npw, int(1.02 * (ws + proj + pot + tables + vectors)) + (8 << 20)


def solve_one(w, prec, device=0, torch=None):
    """One request on a fresh context and stream; returns a result dict.  The
    context is closed whatever happens (a failed solve raises after that)."""
    if torch is None:
        import torch
    from .solver import PlaneWaveProblem
    t0 = time.perf_counter()
    stream = torch.cuda.Stream(device)
    prob = PlaneWaveProblem.from_workload(w, device=device, stream=stream, prec=prec)
    try:
        t1 = time.perf_counter()
        eig, X, status = prob.solve(w.tol, max_iter=300, allow_not_converged=True)
        res = prob.ctx.get_residuals(w.nbands)
        st = prob.ctx.get_stats()
        stream.synchronize()
        t2 = time.perf_counter()
        out = {"name": w.name, "npw": prob.npw, "nbands": w.nbands, "prec": int(prec),
               "eig": eig, "max_residual": float(res.max()),
               "converged": status != PW_ERR_NOT_CONVERGED,
               "iterations": st["iterations"], "setup_s": t1 - t0, "solve_s": t2 - t1}
        del X
    finally:
        prob.ctx.close()
    del prob
    return out


class Server:
    """Admission control and continuous batching over independent solves."""

    def __init__(self, device=0, budget_bytes=None, max_active=8, log=None, solve=None):
        import torch
        self.torch = torch
        self.solve = solve_one if solve is None else solve   # (w, prec, device, torch) -> dict
        self.device = device
        self.log = log   # optional callable taking one line per finished request
        if budget_bytes is None:
            free, _total = torch.cuda.mem_get_info(device)
            budget_bytes = int(0.8 * free)
        self.budget = budget_bytes
        self.max_active = max_active

    def run(self, requests):
        """requests: list of (arrival_seconds, workload, prec).  Returns the
        per-request results (in request order) and a summary."""
        order = sorted(range(len(requests)), key=lambda i: requests[i][0])
        sizes = [footprint(w, prec)[1] for _, w, prec in requests]
        for i, b in enumerate(sizes):
            if b > self.budget:
                raise ValueError(f"request {i} needs {b} bytes, more than the budget {self.budget}")
        lock = threading.Condition()
        pending = collections.deque()
        state = {"used": 0, "active": 0, "done": 0}
        results = [None] * len(requests)
        t0 = time.perf_counter()

        def worker(i):
            _, w, prec = requests[i]
            r = {"name": w.name, "nbands": w.nbands, "prec": int(prec), "eig": None,
                 "max_residual": float("inf"), "converged": False, "solve_s": float("nan")}
            err = "interrupted"
            try:
                r = self.solve(w, prec, self.device, self.torch)
                err = None
            except Exception as exc:          # a failed request releases its slot too
                err = f"{type(exc).__name__}: {exc}"
            finally:
                with lock:
                    results[i].update(r)
                    results[i]["error"] = err
                    results[i]["done_s"] = time.perf_counter() - t0
                    state["used"] -= sizes[i]
                    state["active"] -= 1
                    state["done"] += 1
                    lock.notify_all()
            if self.log:
                what = f"solve {r['solve_s']:.2f} s" if err is None else f"failed ({err})"
                self.log(f"request {i}: {r['nbands']} bands, {what}, latency "
                         f"{results[i]['done_s'] - results[i]['arrival_s']:.2f} s")

        threads = []
        nxt = 0
        with lock:
            while state["done"] < len(requests):
                now = time.perf_counter() - t0
                while nxt < len(order) and requests[order[nxt]][0] <= now:
                    pending.append(order[nxt])
                    nxt += 1
                # admit, oldest first, while a slot is free and the footprint fits
                while (pending and state["active"] < self.max_active
                       and state["used"] + sizes[pending[0]] <= self.budget):
                    i = pending.popleft()
                    state["used"] += sizes[i]
                    state["active"] += 1
                    results[i] = {"arrival_s": requests[i][0], "admitted_s": now,
                                  "footprint_bytes": sizes[i]}
                    th = threading.Thread(target=worker, args=(i,), daemon=True)
                    th.start()
                    threads.append(th)
                wait = None
                if nxt < len(order):
                    wait = max(0.0, requests[order[nxt]][0] - (time.perf_counter() - t0))
                lock.wait(timeout=wait if wait is not None else 1.0)
        for th in threads:
            th.join()
        lat = np.array([r["done_s"] - r["arrival_s"] for r in results])
        span = max(r["done_s"] for r in results) - min(r["arrival_s"] for r in results)
        summary = {"requests": len(requests), "solves_per_s": len(requests) / span,
                   "eigenpairs_per_s": sum(r["nbands"] for r in results) / span,
                   "latency_p50_s": float(np.percentile(lat, 50)),
                   "latency_p99_s": float(np.percentile(lat, 99)),
                   "max_wait_s": float(max(r["admitted_s"] - r["arrival_s"] for r in results)),
                   "failed": sum(r["error"] is not None for r in results),
                   "all_converged": all(r["converged"] for r in results),
                   "max_residual": max(r["max_residual"] for r in results)}
        return results, summary


def poisson_arrivals(n, rate, seed=4):
    """Arrival times of n requests at `rate` per second (exponential gaps, seeded)."""
    gaps = np.random.default_rng(seed).exponential(1.0 / rate, n)
    return np.cumsum(gaps) - gaps[0]


def main():
    from workloads import make_request
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=16)
    ap.add_argument("--rate", type=float, default=2.0, help="arrivals per second")
    ap.add_argument("--max-active", type=int, default=8)
    ap.add_argument("--lmax", type=float, default=24.0)
    ap.add_argument("--ecut-max", type=float, default=25.0)
    args = ap.parse_args()
    arr = poisson_arrivals(args.requests, args.rate)
    reqs = []
    for i in range(args.requests):
        w, mixed = make_request(i, L_range=(8.0, args.lmax), ecut_range=(5.0, args.ecut_max))
        reqs.append((float(arr[i]), w, PW_PREC_MIXED if mixed else PW_PREC_FP64))
    srv = Server(max_active=args.max_active, log=lambda line: print(f"[serve] {line}", file=sys.stderr, flush=True))
    _, summary = srv.run(reqs)
    print(json.dumps(summary))


if __name__ == "__main__":
    main()
