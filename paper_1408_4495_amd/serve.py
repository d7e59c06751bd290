"""Continuous-batching request loop over the C ABI.

Requests (n, d, w, medium, incident directions) arrive over time.  A request
is admitted as soon as a worker slot is free and its exact device footprint
(problem workspace + solve workspace for its right-hand sides + its fields,
from lsp_plan_bytes) fits in the remaining HBM budget; admitted requests run
concurrently, each on its own HIP stream, so their kernels overlap on the
GPU.  Set-up, factorisation and Krylov state stay on the device for the
request's lifetime and are released when it completes.  The library calls
release the GIL (ctypes), so worker threads drive the GPU in parallel.

Every kernel is deterministic and independent of what else runs, so a
request's result is bit-identical alone and in the mix.
"""
import threading
import time

import numpy as np

from . import lsp


class Request:
    def __init__(self, rid, n, d, omega, m, uI, arrival):
        self.id, self.n, self.d, self.omega = rid, n, d, float(omega)
        self.m = np.asarray(m, dtype=np.float64)
        self.uI = np.atleast_2d(np.asarray(uI, dtype=np.complex128))
        self.arrival = float(arrival)
        self.admit = self.start = self.finish = None
        self.u = None
        self.info = None
        self.status = None
        self.footprint = 0

    @property
    def nrhs(self):
        return self.uI.shape[0]


class Server:
    """Admission by HBM footprint, `slots` concurrent requests on their own streams."""

    def __init__(self, device="cuda:0", precision="mixed", slots=4, hbm_budget=None, tol=1e-8,
                 keep_results=True):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        lsp.load()
        self.precision = precision
        self.slots = slots
        self.tol = tol
        self.keep = keep_results
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info(self.device)
            hbm_budget = int(0.9 * free)
        self.budget = int(hbm_budget)
        self.plans = {}
        self.lock = threading.Lock()
        self.cv = threading.Condition(self.lock)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(slots)]

    def plan(self, n, d):
        key = (n, d)
        with self.lock:
            p = self.plans.get(key)
            if p is None:
                p = lsp.Plan(n, d, max_nrhs=32, precision=self.precision, tol=self.tol)
                self.plans[key] = p
        return p

    def footprint(self, req):
        p = self.plan(req.n, req.d)
        pb, sb = p.bytes(req.nrhs)
        N = req.n ** req.d
        return pb + sb + 2 * req.nrhs * N * 16 + N * 8

    def _run_one(self, req, stream):
        torch = self.torch
        plan = self.plan(req.n, req.d)
        with torch.cuda.device(self.device), torch.cuda.stream(stream):
            m = torch.tensor(req.m, dtype=torch.float64, device=self.device)
            uI = torch.tensor(req.uI, dtype=torch.complex128, device=self.device)
            req.start = time.perf_counter()
            pb = lsp.Problem(plan, req.omega, m, device=self.device, stream=stream)
            pb.factor()
            u, info, st = pb.solve(uI)
            stream.synchronize()
            req.finish = time.perf_counter()
            req.info, req.status = info, st
            if self.keep:
                req.u = u.cpu().numpy()
            del pb, u, m, uI

    def run(self, requests, realtime=True, exclude_first=0, strict=True):
        """Serve `requests` (arrival times in seconds from the start).  Returns
        a report with p50/p99 latency and solves/s over the requests after the
        first `exclude_first` by arrival (all of them are served).  A request
        that fails raises at the end with strict, else it is listed under
        "failed" and left out of the statistics."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        for r in reqs:
            r.footprint = self.footprint(r)
            if r.footprint > self.budget:
                raise ValueError(f"request {r.id} needs {r.footprint} bytes, above the HBM budget {self.budget}")
        t0 = time.perf_counter()
        pending = []          # arrived, not admitted (FIFO by arrival)
        free_slots = list(range(self.slots))
        used = [0]
        done = []
        errors = []
        in_flight = [0]
        peak = [0]
        peak_used = [0]

        def worker(req, slot):
            try:
                self._run_one(req, self.streams[slot])
            except Exception as e:  # reported, never swallowed
                errors.append((req.id, repr(e)))
            with self.cv:
                used[0] -= req.footprint
                free_slots.append(slot)
                in_flight[0] -= 1
                done.append(req)
                self.cv.notify_all()

        i = 0
        threads = []
        with self.cv:
            while len(done) < len(reqs):
                now = time.perf_counter() - t0
                while i < len(reqs) and (not realtime or reqs[i].arrival <= now):
                    pending.append(reqs[i])
                    i += 1
                # admit in arrival order while a slot and memory are free
                while pending and free_slots and used[0] + pending[0].footprint <= self.budget:
                    req = pending.pop(0)
                    slot = free_slots.pop()
                    used[0] += req.footprint
                    peak_used[0] = max(peak_used[0], used[0])
                    in_flight[0] += 1
                    peak[0] = max(peak[0], in_flight[0])
                    req.admit = time.perf_counter()
                    th = threading.Thread(target=worker, args=(req, slot), daemon=True)
                    threads.append(th)
                    th.start()
                if len(done) >= len(reqs):
                    break
                wait = None
                if i < len(reqs) and realtime:
                    wait = max(0.0, reqs[i].arrival - (time.perf_counter() - t0))
                self.cv.wait(timeout=wait if wait is not None else 0.5)
        for th in threads:
            th.join()
        if errors and strict:
            raise RuntimeError(f"requests failed: {errors}")
        failed = {rid for rid, _ in errors}
        meas = reqs[exclude_first:] if exclude_first < len(reqs) else reqs
        meas = [r for r in meas if r.id not in failed]
        ok = [r for r in reqs if r.id not in failed]
        if not meas:
            raise RuntimeError(f"every measured request failed: {errors}")
        start = t0 + meas[0].arrival if realtime else min(r.admit for r in meas)
        makespan = max(r.finish for r in meas) - start
        lat = np.array([r.finish - (t0 + r.arrival if realtime else r.admit) for r in meas])
        solves = sum(r.nrhs for r in meas)
        return {
            "requests": len(meas),
            "solves": solves,
            "makespan_s": makespan,
            "solves_per_s": solves / makespan,
            "latency_ms": {"p50": 1e3 * float(np.percentile(lat, 50)), "p99": 1e3 * float(np.percentile(lat, 99)),
                           "mean": 1e3 * float(lat.mean())},
            "peak_concurrency": peak[0],
            "peak_admitted_bytes": peak_used[0],
            "hbm_budget_bytes": self.budget,
            "all_converged": not failed and all(r.status == 0 and all(x["converged"] for x in r.info) for r in reqs),
            "max_iters": max(max(x["iters"] for x in r.info) for r in ok),
            "failed": sorted(errors),
        }


def requests_from_synth(specs):
    """Wrap synth.serving_requests() dicts as Request objects."""
    return [Request(s["id"], s["n"], s["d"], s["omega"], s["m"], s["uI"], s["arrival"]) for s in specs]


def capacity(server, reqs):
    """Solves/s when the same requests run back to back on one slot (used to
    set an arrival rate as a fraction of capacity)."""
    t0 = time.perf_counter()
    for r in reqs:
        server._run_one(r, server.streams[0])
    el = time.perf_counter() - t0
    return sum(r.nrhs for r in reqs) / el, len(reqs) / el


def main():
    import argparse
    import json
    import sys
    import os
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import synth

    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--rho", type=float, default=0.8)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--precision", default="mixed")
    ap.add_argument("--max-rhs", type=int, default=32)
    args = ap.parse_args()
    srv = Server(precision=args.precision, slots=args.slots, keep_results=False)
    warm = requests_from_synth(synth.serving_requests(args.warmup, 1.0, seed=99, max_rhs=args.max_rhs))
    sps, rps = capacity(srv, warm)
    specs = synth.serving_requests(args.requests, args.rho * rps, seed=5, max_rhs=args.max_rhs)
    rep = srv.run(requests_from_synth(specs))
    rep["capacity_requests_per_s"] = rps
    rep["rho"] = args.rho
    print(json.dumps(rep))


if __name__ == "__main__":
    main()
