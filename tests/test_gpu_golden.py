"""GPU results at the full workload sizes against stored oracle results.

The golden files under tests/golden/ were written by make_golden.py, which
calls only the oracle (numpy/scipy FP64: dense SVD stencils, SuperLU, its own
GMRES) and the seeded input generators.  Compared here:
  * every stencil class's singular values (1e-9 relative) and alpha, C
    (entrywise 1e-9, same phase convention) at 2D n = 256, 1024 and 3D n = 64
    (Section 3.1, eq:Fmin / eq:Emin / eq:Cmin and the 3D sets);
  * the end-to-end solve (Section 3.3) of the 2D n = 1024 workload (40 disks,
    16 plane waves) and of the 3D n = 32 workload (6 bumps, 8 directions),
    in the benchmark's launch configuration (all right-hand sides in one
    batch): FP64 solution within 1e-8 of the oracle's (relative, on a fixed
    strided sample of entries, and the norms), iterations within 1; the
    mixed path's true residual <= 1e-8 and its solution within 1e-6;
  * the same for Section 5's Laplace equation with a potential at 3D n = 48
    (negative Gaussian and smoothed-ball potentials, one delta source, g = K f).
"""
import json
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _lsp():
    import torch
    from paper_1408_4495_amd import lsp
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lsp.load()
    return lsp, torch


def _cplx(pairs):
    a = np.asarray(pairs, dtype=np.float64)
    return a[:, 0] + 1j * a[:, 1]


@pytest.mark.parametrize("name", ["stencils_2d_n256.json", "stencils_2d_n1024.json", "stencils_3d_n64.json"])
def test_stencils_full_size(name):
    g = _load(name)
    n, d, omega = g["n"], g["d"], g["omega"]
    lsp, torch = _lsp()
    plan = lsp.Plan(n, d, buffer_b=g["b"])
    pb = lsp.Problem(plan, omega, np.zeros(n ** d))
    alpha, sigma, C = pb.stencils()
    for cl in g["classes"]:
        c = cl["c"]
        off = np.asarray(cl["offsets"])
        sl = np.sum((off + 1) * (3 ** np.arange(d)), axis=1)
        sig = np.asarray(cl["sigma"])
        s = sig.size
        assert np.all(np.abs(sigma[c, :s] - sig) <= 1e-9 * sig + 1e-15 * sig[0]), (c, sigma[c, :s], sig)
        a_ref, C_ref = _cplx(cl["alpha"]), _cplx(cl["C"])
        assert np.max(np.abs(alpha[c, sl] - a_ref)) <= 1e-9, c
        assert np.max(np.abs(C[c, sl] - C_ref)) <= 1e-9 * np.max(np.abs(C_ref)), c


def _end_to_end(key, golden):
    g = _load(golden)
    w = synth.workload(key)
    n, d, omega, m, uI = w["n"], w["d"], w["omega"], w["m"], w["uI"]
    assert (n, d) == (g["n"], g["d"]) and abs(omega - g["omega"]) < 1e-12
    lsp, torch = _lsp()
    nrhs = uI.shape[0]
    idx = np.arange(g["sample_start"], n ** d, g["sample_stride"])
    out = {}
    for prec in ("fp64", "mixed"):
        plan = lsp.Plan(n, d, max_nrhs=nrhs, precision=prec, buffer_b=g["b"], restart=g["restart"], tol=g["tol"])
        pb = lsp.Problem(plan, omega, m)
        pb.factor()
        u, info, st = pb.solve(uI)
        assert st == 0, info
        u = u.cpu().numpy()
        print(f"{key} {prec}: iters {[i['iters'] for i in info]} oracle {[r['iters'] for r in g['rhs']]}", flush=True)
        for r in range(nrhs):
            ref = g["rhs"][r]
            us = u[r, idx]
            rs = _cplx(ref["u_sample"])
            err = np.linalg.norm(us - rs) / np.linalg.norm(rs)
            nerr = abs(np.linalg.norm(u[r]) - ref["u_norm"]) / ref["u_norm"]
            assert info[r]["converged"] and info[r]["relres_true"] <= 1e-8, (prec, r, info[r])
            if prec == "fp64":
                assert err <= 1e-8 and nerr <= 1e-8, (r, err, nerr)
                assert abs(info[r]["iters"] - ref["iters"]) <= 1, (r, info[r]["iters"], ref["iters"])
            else:
                assert err <= 1e-6 and nerr <= 1e-6, (r, err, nerr)
        out[prec] = u
        del pb
        torch.cuda.empty_cache()
    return out


def test_2d_n1024_16rhs_vs_oracle():
    _end_to_end("c3", "c3_oracle.json")


def test_3d_n32_8rhs_vs_oracle():
    _end_to_end("c4s", "c4s_oracle.json")


def _laplace_end_to_end(key, golden):
    """Section 5's Laplace equation with a potential at 3D n=48: (I + K V) u =
    K f solved on the GPU against the oracle's stored solution."""
    g = _load(golden)
    w = synth.workload(key)
    n, V, f = w["n"], w["V"], w["f"]
    assert (n, 3) == (g["n"], g["d"]) and g["omega"] == 0.0
    lsp, torch = _lsp()
    idx = np.arange(g["sample_start"], n ** 3, g["sample_stride"])
    for prec in ("fp64", "mixed"):
        plan = lsp.Plan(n, 3, max_nrhs=f.shape[0], equation="laplace", precision=prec, buffer_b=g["b"],
                        restart=g["restart"], tol=g["tol"])
        pb = lsp.Problem(plan, 0.0, V)
        pb.factor()
        u, info, st = pb.solve(f, kind="source")
        assert st == 0, info
        u = u.cpu().numpy()
        print(f"{key} {prec}: iters {[i['iters'] for i in info]} oracle {[r['iters'] for r in g['rhs']]}", flush=True)
        for r, ref in enumerate(g["rhs"]):
            rs = _cplx(ref["u_sample"])
            err = np.linalg.norm(u[r, idx] - rs) / np.linalg.norm(rs)
            nerr = abs(np.linalg.norm(u[r]) - ref["u_norm"]) / ref["u_norm"]
            assert info[r]["converged"] and info[r]["relres_true"] <= 1e-8, (prec, r, info[r])
            if prec == "fp64":
                assert err <= 1e-8 and nerr <= 1e-8, (r, err, nerr)
                assert abs(info[r]["iters"] - ref["iters"]) <= 1, (r, info[r]["iters"], ref["iters"])
            else:
                assert err <= 1e-6 and nerr <= 1e-6, (r, err, nerr)
        del pb
        torch.cuda.empty_cache()


def test_3d_n48_laplace_gauss_vs_oracle():
    _laplace_end_to_end("l2", "l2_oracle.json")


def test_3d_n48_laplace_ball_vs_oracle():
    _laplace_end_to_end("l2b", "l2b_oracle.json")
