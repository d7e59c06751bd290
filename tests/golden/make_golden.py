"""Writes the oracle golden files under tests/golden/.

Calls only the oracle and the seeded input generators; nothing here runs or
reads the GPU library.  Targets (one per run, any number on the command line):

  c1        2D n=32 single bump: iterations, residual, sigma_min, k_0, |u|
  st256     stencils (every class's singular values, alpha, C) at 2D n=256
  c3        2D n=1024, 40 disks, 16 plane waves: stencils at n=1024 and, per
            right-hand side, the FP64 GMRES iteration count, residual, |u| and
            a strided sample of u
  c4        3D n=64, 6 bumps, 8 directions: stencils at 3D n=64, and the same
            per-right-hand-side record when the sparse LU fits
  c4s       3D n=32, the same medium recipe and directions (the 3D end-to-end
            golden used when the n=64 sparse LU is out of reach)
  l2, l2b   Section 5's Laplace equation at 3D n=48 (Gaussian / smoothed-ball
            potential, delta source): iterations, residual, |u| and a strided
            sample of u

Usage: python tests/golden/make_golden.py c1 st256 c3 c4s
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle.greens import kernel_table  # noqa: E402
from oracle.stencil import all_stencils  # noqa: E402
from oracle.solve import OracleProblem  # noqa: E402

SAMPLE_STRIDE = {1024: 2055, 64: 517, 32: 67, 48: 113}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _dump(name, obj):
    path = os.path.join(HERE, name)
    with open(path, "w") as f:
        json.dump(obj, f, indent=0)
    log(f"wrote {path}")


def stencil_record(sts, n, d, omega, b):
    return {
        "n": n, "d": d, "omega": omega, "b": b,
        "classes": [{"c": int(st.c), "offsets": st.offsets.tolist(),
                     "sigma": [float(s) for s in st.sigma],
                     "alpha": [[float(a.real), float(a.imag)] for a in st.alpha],
                     "C": [[float(a.real), float(a.imag)] for a in st.C]} for st in sts],
    }


def solve_record(prob, uI, stride):
    out = []
    N = prob.n ** prob.d
    idx = np.arange(0, N, stride)
    for r in range(uI.shape[0]):
        t0 = time.perf_counter()
        res = prob.solve(uI[r])
        log(f"  rhs {r}: iters {res.iters} relres {res.relres:.3e} ({time.perf_counter() - t0:.1f} s)")
        u = res.x
        out.append({"iters": int(res.iters), "relres": float(res.relres),
                    "u_norm": float(np.linalg.norm(u)),
                    "u_sample": [[float(v.real), float(v.imag)] for v in u[idx]]})
    return {"sample_start": 0, "sample_stride": int(stride), "rhs": out}


def make_c1():
    w = synth.workload("c1")
    prob = OracleProblem(w["n"], w["d"], w["omega"], w["m"], b=2)
    res = prob.solve(w["uI"][0])
    out = {
        "workload": "2D n=32 omega=8pi single Gaussian bump, b=2, tol 1e-8, restart 30",
        "iters": res.iters,
        "relres": res.relres,
        "sigma_min": [st.sigma_min for st in prob.stencils],
        "k0": [prob.ktab[0, 0].real, prob.ktab[0, 0].imag],
        "u_norm": float(abs(res.x @ res.x.conj()) ** 0.5),
    }
    with open(os.path.join(HERE, "c1_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)


def make_st256():
    n, d = 256, 2
    omega = 2 * np.pi * n / 8
    t0 = time.perf_counter()
    sts = all_stencils(kernel_table(n, d, omega), d, n, 2)
    log(f"stencils 2D n=256: {time.perf_counter() - t0:.1f} s")
    _dump("stencils_2d_n256.json", stencil_record(sts, n, d, omega, 2))


def _full(key, stencil_name, solve_name, workload=None):
    w = workload or synth.workload(key)
    n, d, omega = w["n"], w["d"], w["omega"]
    t0 = time.perf_counter()
    prob = OracleProblem(n, d, omega, w["m"], b=2)
    log(f"{key}: oracle set-up + SuperLU {time.perf_counter() - t0:.1f} s, "
        f"LU nnz {prob.P.lu.L.nnz + prob.P.lu.U.nnz}")
    if stencil_name:
        _dump(stencil_name, stencil_record(prob.stencils, n, d, omega, 2))
    rec = {"workload": key, "n": n, "d": d, "omega": omega, "b": 2, "tol": 1e-8, "restart": 30}
    rec.update(solve_record(prob, w["uI"], SAMPLE_STRIDE[n]))
    _dump(solve_name, rec)


def make_c3():
    _full("c3", "stencils_2d_n1024.json", "c3_oracle.json")


def make_c4_stencils():
    w = synth.workload("c4")
    n, d, omega = w["n"], w["d"], w["omega"]
    t0 = time.perf_counter()
    sts = all_stencils(kernel_table(n, d, omega), d, n, 2)
    log(f"stencils 3D n=64: {time.perf_counter() - t0:.1f} s")
    _dump("stencils_3d_n64.json", stencil_record(sts, n, d, omega, 2))


def make_c4():
    _full("c4", None, "c4_oracle.json")


def make_c4s():
    _full("c4s", None, "c4s_oracle.json", synth.workload("c4s"))


def make_laplace(key):
    w = synth.workload(key)
    n = w["n"]
    t0 = time.perf_counter()
    prob = OracleProblem(n, 3, 0.0, None, b=2, potential=w["V"])
    log(f"{key}: oracle set-up + SuperLU {time.perf_counter() - t0:.1f} s")
    idx = np.arange(0, n ** 3, SAMPLE_STRIDE[n])
    out = []
    for r in range(w["f"].shape[0]):
        res = prob.solve_source(w["f"][r])
        log(f"  source {r}: iters {res.iters} relres {res.relres:.3e}")
        out.append({"iters": int(res.iters), "relres": float(res.relres), "u_norm": float(np.linalg.norm(res.x)),
                    "u_sample": [[float(v.real), float(v.imag)] for v in res.x[idx]]})
    _dump(f"{key}_oracle.json", {"workload": key, "n": n, "d": 3, "omega": 0.0, "b": 2, "tol": 1e-8,
                                 "restart": 30, "sample_start": 0, "sample_stride": SAMPLE_STRIDE[n], "rhs": out})


TARGETS = {"c1": make_c1, "st256": make_st256, "c3": make_c3, "st3d64": make_c4_stencils,
           "c4": make_c4, "c4s": make_c4s, "l2": lambda: make_laplace("l2"), "l2b": lambda: make_laplace("l2b")}

if __name__ == "__main__":
    for t in sys.argv[1:] or ["c1"]:
        TARGETS[t]()
