"""Continuous-batching request loop for CCSD solves on one GPU.

Requests of different (nocc, nvir, naux) arrive over time (Poisson process).
A request is admitted as soon as a slot is free and its a-priori device
footprint (exacc_ccsd_memory_estimate) fits in what is left of the HBM budget;
otherwise it waits in FIFO order.  Every admitted request owns one exacc handle
on its own HIP stream, driven by its own host thread: its iterations
interleave with those of every other active request and their kernels overlap
on the device.  On convergence the handle is destroyed, its memory returns to
the budget and waiting requests are admitted.  Per request the loop records
arrival, admission, start and finish times; the report gives p50/p99 latency
(finish - arrival) and solves per second.

    python -m paper_2103_08473_amd.serve --requests 64 --rate 2.0
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import math
import multiprocessing
import threading
import time
from dataclasses import dataclass, field

import numpy as np

from . import exacc
from .synth import make_system, serving_request


@dataclass
class Request:
    k: int
    nocc: int
    nvir: int
    naux: int
    seed: int
    arrival: float = 0.0
    admitted: float = math.nan
    finished: float = math.nan
    energy: complex = 0j
    iterations: int = 0
    device_ms: float = 0.0
    converged: bool = False
    status: int = 0
    mem: int = 0
    mem_wait: bool = False   # was at the head of the queue with a slot free but not the memory
    error: str = ""
    inputs: object = field(default=None, repr=False)


def _make_inputs(shape):
    nocc, nvir, naux, seed = shape
    return make_system(nocc, nvir, naux, seed=seed)


def solve_one(req: Request, opts: dict):
    """Run one request to convergence on a fresh handle (own stream)."""
    eps, B = req.inputs
    with exacc.CCSD(eps, B, req.nocc, **opts) as cc:
        it = 0
        conv = False
        st = 0
        while it < opts.get("max_iter", 60):
            st, n, r, conv = cc.iterate(1)
            it += n
            if conv or st == exacc.ERR_DIVERGED:
                break
        req.energy = cc.energy()
        if opts.get("timing"):   # HIP-event time of the request's stages on its own stream
            req.device_ms = float(sum(cc.stage_times().values()))
    req.iterations, req.converged, req.status = it, conv, st
    return req


class Server:
    def __init__(self, hbm_budget: int, max_active: int, opts: dict, progress=None):
        self.progress = progress
        self.budget = hbm_budget
        self.max_active = max_active
        self.opts = dict(opts)
        self.lock = threading.Condition()
        self.in_use = 0
        self.active = 0
        self.queue: list[Request] = []
        self.done: list[Request] = []
        self.pool = cf.ThreadPoolExecutor(max_workers=max_active)
        self.t0 = time.perf_counter()

    def now(self):
        return time.perf_counter() - self.t0

    def submit(self, req: Request):
        req.mem = exacc.memory_estimate(req.nocc, req.nvir, req.naux,
                                        precision=self.opts.get("precision", exacc.FP64))
        if req.mem > self.budget:
            req.status, req.error = exacc.ERR_NOMEM, "request exceeds the whole HBM budget"
            req.finished = self.now()
            with self.lock:
                self.done.append(req)
            return
        with self.lock:
            self.queue.append(req)
            self._admit_locked()

    def _admit_locked(self):
        while self.queue and self.active < self.max_active and \
                self.in_use + self.queue[0].mem <= self.budget:
            req = self.queue.pop(0)
            self.active += 1
            self.in_use += req.mem
            req.admitted = self.now()
            self.pool.submit(self._run, req)
        if self.queue and self.active < self.max_active:
            self.queue[0].mem_wait = True

    def _run(self, req: Request):
        try:
            solve_one(req, self.opts)
        except Exception as e:  # recorded, not raised: the loop keeps serving
            req.error = str(e)
            req.status = getattr(e, "status", exacc.ERR_DEVICE)
        req.finished = self.now()
        req.inputs = None
        if self.progress:
            self.progress("done %d (%d, %d, %d) it %d latency %.2fs" % (
                req.k, req.nocc, req.nvir, req.naux, req.iterations, req.finished - req.arrival))
        with self.lock:
            self.active -= 1
            self.in_use -= req.mem
            self.done.append(req)
            self._admit_locked()
            self.lock.notify_all()

    def drain(self, n_total: int):
        with self.lock:
            while len(self.done) < n_total:
                self.lock.wait(timeout=1.0)
        self.pool.shutdown(wait=True)


def run_stream(requests: list[Request], rate: float, hbm_budget: int, max_active: int,
               opts: dict, producers: int = 8, progress=None):
    """Feed the requests at Poisson arrival times (rate per second) and serve them."""
    rng = np.random.default_rng(12345)
    gaps = rng.exponential(1.0 / rate, len(requests)) if rate > 0 else np.zeros(len(requests))
    arrivals = np.cumsum(gaps)
    # input generation in spawned processes (no fork of a process that may hold the GPU)
    gen = cf.ProcessPoolExecutor(max_workers=producers, mp_context=multiprocessing.get_context("spawn"))
    futs = [gen.submit(_make_inputs, (r.nocc, r.nvir, r.naux, r.seed)) for r in requests]
    srv = Server(hbm_budget, max_active, opts, progress=progress)
    for req, t_arr, fut in zip(requests, arrivals, futs):
        req.inputs = fut.result()                   # inputs exist before the request "arrives"
        delay = t_arr - srv.now()
        if delay > 0:
            time.sleep(delay)
        req.arrival = srv.now()
        srv.submit(req)
        if progress:
            progress("arrived %d (%d, %d, %d)" % (req.k, req.nocc, req.nvir, req.naux))
    srv.drain(len(requests))
    gen.shutdown()
    return srv


def report(reqs: list[Request], makespan: float):
    ok = [r for r in reqs if r.converged]
    lat = np.array([r.finished - r.arrival for r in ok])
    wait = np.array([r.admitted - r.arrival for r in ok])
    return {
        "requests": len(reqs),
        "converged": len(ok),
        "failed": [(r.k, r.status, r.error) for r in reqs if not r.converged],
        "makespan_s": round(makespan, 3),
        "solves_per_s": round(len(ok) / makespan, 4) if makespan > 0 else None,
        "latency_p50_s": round(float(np.percentile(lat, 50)), 4) if lat.size else None,
        "latency_p99_s": round(float(np.percentile(lat, 99)), 4) if lat.size else None,
        "queue_wait_p50_s": round(float(np.percentile(wait, 50)), 4) if wait.size else None,
        "mean_iterations": round(float(np.mean([r.iterations for r in ok])), 2) if ok else None,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=64)
    ap.add_argument("--first", type=int, default=0, help="index of the first request of the stream")
    ap.add_argument("--out", default=None, help="write per-request records (JSON) here")
    ap.add_argument("--rate", type=float, default=2.0, help="Poisson arrival rate, requests/s")
    ap.add_argument("--max-active", type=int, default=8)
    ap.add_argument("--hbm-budget-gb", type=float, default=200.0)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--precision", choices=["fp64", "mixed", "bf16x3"], default="mixed")
    ap.add_argument("--check-alone", type=int, default=4,
                    help="re-solve this many requests (the smallest) alone and compare energies bitwise")
    args = ap.parse_args()
    prec = {"mixed": exacc.MIXED_FP32, "bf16x3": exacc.MIXED_BF16X3, "fp64": exacc.FP64}[args.precision]
    opts = dict(precision=prec, tol=args.tol, max_iter=80)
    reqs = []
    for k in range(args.first, args.first + args.requests):
        o, v, X, seed = serving_request(k)
        reqs.append(Request(k, o, v, X, seed))
    t0 = time.perf_counter()
    srv = run_stream(reqs, args.rate, int(args.hbm_budget_gb * (1 << 30)), args.max_active, opts,
                     progress=lambda m: print(m, flush=True))
    makespan = time.perf_counter() - t0
    out = report(srv.done, makespan)
    out.update({"first": args.first, "rate_per_s": args.rate, "max_active": args.max_active,
                "hbm_budget_gb": args.hbm_budget_gb, "precision": args.precision, "tol": args.tol})
    # each result alone vs in the mix
    same = []
    for r in sorted(srv.done, key=lambda r: (r.nvir, r.k))[:args.check_alone]:
        alone = Request(r.k, r.nocc, r.nvir, r.naux, r.seed)
        alone.inputs = _make_inputs((r.nocc, r.nvir, r.naux, r.seed))
        solve_one(alone, opts)
        same.append({"k": r.k, "bitwise_equal": alone.energy == r.energy,
                     "abs_diff": abs(alone.energy - r.energy)})
    out["alone_vs_mix"] = same
    if args.out:
        recs = [{"k": r.k, "nocc": r.nocc, "nvir": r.nvir, "naux": r.naux, "arrival": r.arrival,
                 "admitted": r.admitted, "finished": r.finished, "iterations": r.iterations,
                 "converged": r.converged, "energy": [r.energy.real, r.energy.imag]}
                for r in sorted(srv.done, key=lambda r: r.k)]
        with open(args.out, "w") as f:
            json.dump({"summary": out, "requests": recs}, f)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
