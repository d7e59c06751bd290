"""Benchmark of the sparsifying-preconditioned Lippmann-Schwinger solve on one GPU.

One step = one pass of the whole hot path over one batch of right-hand sides:
set-up on the GPU (kernel table, Green's spectrum, stencil null vectors,
matrix M), multifrontal factorisation, and preconditioned GMRES to a true
relative residual of 1e-8 for every right-hand side.  The symbolic plan
(nested dissection of the grid graph, a function of n and d only) is built
once outside the timed region; inputs are resident in HBM before timing.

The reported value is solves per second (one solve = one incident direction
driven to 1e-8) of the mixed-precision path; the complex128 path is timed on
the same workload and reported beside it.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD_TEXT = {
    "c1": "2D n=32 (N=1024), omega=8pi, one Gaussian bump, 1 plane wave",
    "c2": "2D n=256 (N=65536), omega=64pi (8 pts/wavelength), 8 seeded Gaussian bumps, 1 plane wave",
    "c3": "2D n=1024 (N=1048576), omega=256pi, 40 seeded smoothed disks, 16 plane waves",
    "c4": "3D n=64 (N=262144), omega=16pi, 6 seeded Gaussian bumps, 8 plane waves",
}

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_path(lsp, torch, w, m_dev, u_dev, prec, steps, warmup):
    n, d, omega = w["n"], w["d"], w["omega"]
    nrhs = u_dev.shape[0]
    plan = lsp.Plan(n, d, max_nrhs=nrhs, precision=prec)

    def step():
        pb = lsp.Problem(plan, omega, m_dev)
        pb.factor()
        u, info, st = pb.solve(u_dev)
        return pb, u, info, st

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    lat = []
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    tot0, tot1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    tot0.record()
    for _ in range(steps):
        ev0.record()
        pb, u, info, st = step()
        ev1.record()
        torch.cuda.synchronize()
        lat.append(ev0.elapsed_time(ev1))
    tot1.record()
    torch.cuda.synchronize()
    total_ms = tot0.elapsed_time(tot1)
    if st != 0 or not all(i["converged"] for i in info):
        raise RuntimeError(f"{prec} path failed: status {st}, {info}")
    # phase split (untimed extra step; set-up only enqueues, so it is
    # followed by a synchronisation; factor and solve synchronise themselves)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pb = lsp.Problem(plan, omega, m_dev)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pb.factor()
    t2 = time.perf_counter()
    u2, info2, _ = pb.solve(u_dev)
    t3 = time.perf_counter()
    # solve-only rate with the factorisation cached
    reps = max(3, steps)
    torch.cuda.synchronize()
    s0 = time.perf_counter()
    for _ in range(reps):
        pb.solve(u_dev)
    torch.cuda.synchronize()
    solve_only_s = (time.perf_counter() - s0) / reps
    return {
        "plan": plan, "problem": pb, "u": u2, "info": info2,
        "ms_per_step": total_ms / steps,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "solves_per_s": nrhs / (total_ms / steps / 1000.0),
        "solve_only_solves_per_s": nrhs / solve_only_s,
        "phase_ms": {"setup": 1e3 * (t1 - t0), "factor": 1e3 * (t2 - t1), "solve": 1e3 * (t3 - t2)},
        "iters": [i["iters"] for i in info2],
        "relres_true_max": max(i["relres_true"] for i in info2),
    }


# HBM traffic per launch measured with hardware counters (FETCH_SIZE and
# WRITE_SIZE, scaled by a device-to-device copy of known size); a record is
# used only while the source file of the kernel is unchanged.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_2d_n256.md")
CSRC = os.path.join(ROOT, "paper_1408_4495_amd", "csrc")


def source_sha256(fname):
    import hashlib
    with open(os.path.join(CSRC, fname), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def recorded_traffic(name):
    """(bytes per launch, record) for kernel `name` from the counter summary,
    or (None, reason) when absent or taken on a different kernel source."""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None, "no counter summary"
    marker = "<!-- traffic-json:"
    if marker not in text:
        return None, "no counter summary"
    rec = json.loads(text.split(marker, 1)[1].split("-->", 1)[0])
    k = rec["kernels"].get(name)
    if k is None:
        return None, "kernel not in the counter summary"
    if source_sha256(k["source"]) != k["sha256"]:
        return None, f"{k['source']} changed since the counters were taken"
    return k["bytes_per_launch"], rec


def kernel_model(name, st, w, nrhs):
    """Algorithmic work of one launch of a library kernel, from the plan:
    (bound, amount per launch, unit), amount None where it is summed over the
    launches instead.  Returns None for kernels without a model."""
    esz = 8 if "[c64]" in name else 16
    n, d, N, L, nlev = st["n"], st["d"], st["N"], st["L"], st["nlevels"]
    base = name.split(" ")[0]
    if base in ("fwd", "bwd", "fwd_dense", "bwd_dense"):
        # one sweep reads every L (or U) panel entry and inverted diagonal
        # block of the chain levels, and the formed operators of the dense
        # levels, once per right-hand-side group (one group here), plus the
        # N-vector it consumes and the N-vector it produces, shared out by
        # level; spread over the launches of each kind
        dl = st["dense_levels"]
        lev, entries = (dl, st["dense_entries"]) if base.endswith("_dense") else (nlev - dl, st["sweep_entries"])
        if lev == 0:
            return None
        per_app = entries * esz + 2 * N * esz * nrhs * lev / nlev
        return "hbm", per_app / lev, "GB/s"
    if base == "gemm_update":
        # the plain trailing-update launches (the update launches that also
        # factor a diagonal block, update_lu and panel_step, are bound by
        # that factorisation's latency and carry no separate model)
        return "mfma", None, "TFLOP/s"
    if base == "diag_lu":
        # per 32 x 32 block: complex LU (sum_j (31-j)^2 multiply-adds) and the
        # two triangular inverses (about 32^3/6 multiply-adds each), 8 real
        # flops per complex multiply-add; summed over the plan's panel blocks
        return "alu", None, "TFLOP/s"
    if base.startswith("fft_"):
        lines = {"fft_first": n ** (d - 1), "fft_last": n ** (d - 1)}
        if base in lines:
            # read / write an n-point grid row (complex128 field) and an L-point work row
            per = lines[base] * (n * 16 + L * esz) * nrhs
            return "hbm", per, "GB/s"
        if base == "fft_conv":
            nl = L ** (d - 1)
            return "hbm", nl * 2 * n * esz * nrhs + (n + 1) ** d * esz, "GB/s"
    return None


DIAG_FLOPS_PER_BLOCK = 8.0 * (sum((31 - j) ** 2 for j in range(32)) + 2 * 32 ** 3 / 6.0)


def measure_roofline(lsp, torch, w, m_dev, u_dev, prec):
    """Live per-kernel timing (HIP events on the kernel's stream) over one
    extra step; returns the roofline record of the kernel with the most time
    (among those with a work model) and the per-kernel table."""
    n, d, omega = w["n"], w["d"], w["omega"]
    nrhs = u_dev.shape[0]
    plan = lsp.Plan(n, d, max_nrhs=nrhs, precision=prec)
    st = plan.stats()
    torch.cuda.synchronize()
    lsp.timing_reset()
    lsp.timing_enable(True)
    try:
        pb = lsp.Problem(plan, omega, m_dev)
        pb.factor()
        pb.solve(u_dev)
        torch.cuda.synchronize()
    finally:
        lsp.timing_enable(False)
    times = lsp.timing_read()
    ranked = sorted(times.items(), key=lambda kv: -kv[1][0])
    total = sum(v[0] for v in times.values())
    table = {k: {"ms": round(v[0], 4), "launches": v[1], "avg_us": round(1e3 * v[0] / v[1], 3)}
             for k, v in ranked[:12]}
    for name, (ms, cnt) in ranked:
        model = kernel_model(name, st, w, nrhs)
        if model is None:
            continue
        bound, per_launch, unit = model
        avg_s = ms / cnt / 1e3
        fp64 = "[c64]" not in name
        if bound == "mfma":
            # the update flops of one factorisation outside the launches
            # that also factor a diagonal block
            flops = st["update_flops"] - st["fused_update_flops"]
            achieved = flops / (ms / 1e3) / 1e12
            peak = 78.6 if fp64 else 157.3      # dense FP64 / FP32 matrix cores
            amount = flops / cnt
        elif bound == "alu":
            flops = DIAG_FLOPS_PER_BLOCK * (st["panel_blocks"] - st["fused_blocks"])
            achieved = flops / (ms / 1e3) / 1e12
            peak = 78.6 if fp64 else 157.3      # FP64 / FP32 vector ALUs
            amount = flops / cnt
        else:
            achieved = per_launch / avg_s / 1e9
            peak = HBM_PEAK_GBS
            amount = per_launch
        traffic, rec = recorded_traffic(name)
        out = {"kernel": name, "bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
               "frac": achieved / peak, "traffic": traffic, "avg_launch_us": 1e6 * avg_s,
               "launches": cnt, "algorithmic_per_launch": amount, "share_of_kernel_time": ms / total}
        if traffic is None:
            out["traffic_note"] = rec
        else:
            out["traffic_note"] = (f"HBM bytes per launch from rocprofv3 FETCH_SIZE x {rec['fetch_scale']:.3f} + "
                                   f"WRITE_SIZE x {rec['write_scale']:.3f} (copy-calibrated), {rec['command']}")
        return out, table
    return None, table


def cpu_baseline(w, budget_s=12.0):
    """The oracle (numpy/scipy, FP64) on the host cores: set-up, SuperLU
    factorisation and GMRES for the first right-hand side, repeated until the
    time budget is used."""
    from oracle.solve import OracleProblem
    cores = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    done = 0
    while True:
        prob = OracleProblem(w["n"], w["d"], w["omega"], w["m"])
        res = prob.solve(w["uI"][0])
        done += 1
        if time.perf_counter() - t0 >= budget_s or done >= 12:
            break
    el = time.perf_counter() - t0
    return {"value": done / el, "unit": "solves/s", "cores": cores, "kind": "oracle",
            "sample": f"{done} full oracle solve(s) (set-up + SuperLU + GMRES) of the first right-hand side "
                      f"of the same workload, {el:.1f} s; numpy/scipy, SuperLU and numpy.fft single-threaded, "
                      f"LAPACK SVD multi-threaded; iterations {res.iters}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("this benchmark runs on one GPU only: the solver has no multi-GPU path "
              "(right-hand sides and requests would shard across GPUs with no exchange)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_1408_4495_amd import lsp

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    lsp.load()
    w = synth.workload(args.workload)
    dev = torch.device("cuda:0")
    m_dev = torch.tensor(w["m"], dtype=torch.float64, device=dev)
    u_dev = torch.tensor(w["uI"], dtype=torch.complex128, device=dev)
    nrhs = u_dev.shape[0]

    log(f"[bench] workload {args.workload}: {WORKLOAD_TEXT[args.workload]}")
    res = {}
    for prec in ("fp64", "mixed"):
        log(f"[bench] path {prec}: warmup {args.warmup}, steps {args.steps}")
        res[prec] = run_path(lsp, torch, w, m_dev, u_dev, prec, args.steps, args.warmup)
        r = res[prec]
        log(f"[bench] {prec}: {r['ms_per_step']:.2f} ms/step, iters {r['iters']}, "
            f"phases {json.dumps({k: round(v, 2) for k, v in r['phase_ms'].items()})}")
    u64 = res["fp64"]["u"]
    umx = res["mixed"]["u"]
    diff = float(torch.linalg.norm(umx - u64) / torch.linalg.norm(u64))

    log("[bench] live kernel timing for the roofline")
    roof, ktable = measure_roofline(lsp, torch, w, m_dev, u_dev, "mixed")
    log(f"[bench] kernel table: {json.dumps(ktable)}")

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        cpu = cpu_baseline(w)

    mx, fp = res["mixed"], res["fp64"]
    out = {
        "metric": "LS solves/sec at 1e-8 rel. residual, mixed vs FP64 path; p50/p99 latency",
        "value": mx["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mx["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64+c128",
        "data": "synthetic (seeded media and plane waves)",
        "config": {"workload": WORKLOAD_TEXT[args.workload], "n": w["n"], "d": w["d"], "nrhs": nrhs,
                   "tol": 1e-8, "restart": 30, "step": "setup + factor + GMRES solve, end to end"},
        "latency_ms": mx["latency_ms"],
        "paths": {
            p: {"solves_per_s": res[p]["solves_per_s"], "ms_per_step": res[p]["ms_per_step"],
                "solve_only_solves_per_s": res[p]["solve_only_solves_per_s"],
                "latency_ms": res[p]["latency_ms"], "phase_ms": res[p]["phase_ms"],
                "iters": res[p]["iters"], "relres_true_max": res[p]["relres_true_max"]}
            for p in ("fp64", "mixed")},
        "mixed_vs_fp64": {"speedup": mx["solves_per_s"] / fp["solves_per_s"], "solution_rel_diff": diff},
        "roofline": roof,
        "kernel_ms": ktable,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
