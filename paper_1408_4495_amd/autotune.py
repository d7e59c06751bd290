"""Autotuner for the frontal factorisation's tile shapes.

For a grid (n, d) and precision it times the multifrontal factorisation
(lsp_factor) of one set-up problem under candidate per-level tile tables
(lsp_plan_set_tiles: 32, 64 or 128 square MFMA tiles for F22 -= L21 U12),
starting from the best uniform table and then changing one level at a time
from the top of the tree while that lowers the median factor time.  The
result is the table a plan for this (n, d) should use; tuning changes speed
only, never what is computed.
"""
import statistics
import time

import numpy as np

from . import lsp

TILES = (32, 64, 128)


def _time_factor(torch, pb, reps):
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pb.factor()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return statistics.median(ts)


def tune_tiles(n, d, precision="mixed", omega=None, m=None, reps=3, device="cuda:0", log=None, cache=None):
    """Return {"tiles": [...], "factor_ms": best, "uniform_ms": {...}, "trials": k};
    with `cache` (a file path) the table is also written there, where plans
    created with tile_cache=path pick it up."""
    import torch
    omega = 2 * np.pi * n / 8 if omega is None else omega
    if m is None:
        rng = np.random.default_rng([14084495, 9, n, d])
        ax = (np.arange(n) + 0.5) / n
        X = np.stack(np.meshgrid(*([ax] * d), indexing="ij"), axis=-1).reshape(-1, d)
        c = rng.uniform(0.3, 0.7, size=d)
        m = 0.2 * np.exp(-np.sum((X - c) ** 2, axis=1) / (2 * 0.1 ** 2))
    plan = lsp.Plan(n, d, precision=precision)
    pb = lsp.Problem(plan, omega, m, device=device)
    nl = plan.stats()["nlevels"]
    trials = 0
    uniform = {}
    for t in TILES:
        plan.set_tiles([t] * nl)
        uniform[t] = _time_factor(torch, pb, reps)
        trials += 1
    best_t = min(uniform, key=uniform.get)
    best = [best_t] * nl
    best_time = uniform[best_t]
    for level in range(nl - 1, -1, -1):
        for t in TILES:
            if t == best[level]:
                continue
            cand = list(best)
            cand[level] = t
            plan.set_tiles(cand)
            tt = _time_factor(torch, pb, reps)
            trials += 1
            if tt < best_time * 0.98:
                best, best_time = cand, tt
        if log:
            log(f"[autotune] n={n} d={d} level {level}: tiles {best} {1e3 * best_time:.3f} ms")
    plan.set_tiles(best)
    if cache is not None:
        plan.save_tiles(cache)
    return {"tiles": best, "factor_ms": 1e3 * best_time,
            "uniform_ms": {str(k): 1e3 * v for k, v in uniform.items()}, "trials": trials}


def main():
    import argparse
    import json
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--d", type=int, default=2)
    ap.add_argument("--precision", default="mixed")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--cache", default=None, help="tile cache file to write the table to")
    args = ap.parse_args()
    print(json.dumps(tune_tiles(args.n, args.d, args.precision, reps=args.reps, cache=args.cache)))


if __name__ == "__main__":
    main()
