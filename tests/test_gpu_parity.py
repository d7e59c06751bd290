"""GPU parity: each step of the HIP path, called through the C ABI, against
the CPU oracle on the same seeded inputs.  Tolerances are relative and are
derived from the arithmetic (FP64 rounding of each step, or FP32 for the
mixed-precision convolution), as listed in each test."""
import numpy as np
import pytest

import synth
from oracle.greens import kernel_table
from oracle.operator import apply_K_direct, Operator, dense_K
from oracle.stencil import all_stencils, slot, class_offsets
from oracle.sparse import build_QM, Preconditioner
from oracle.solve import OracleProblem

pytestmark = pytest.mark.gpu


def _lsp():
    import torch
    from paper_1408_4495_amd import lsp
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lsp.load()
    return lsp, torch


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


def _problem(n, d, omega, m, **kw):
    lsp, torch = _lsp()
    plan = lsp.Plan(n, d, **kw)
    return lsp, torch, plan, lsp.Problem(plan, omega, m)


@pytest.mark.parametrize("n,d", [(32, 2), (256, 2), (16, 3), (48, 2)])
def test_kernel_table(n, d):
    """Own Bessel/Hankel evaluation vs scipy (AMOS): entries agree to 1e-13 of
    max|k| and to 1e-13 relative entrywise (arguments up to 0.79 n sqrt(d);
    measured: about 2e-15 of max|k|)."""
    omega = 2 * np.pi * n / 8
    lsp, torch, plan, pb = _problem(n, d, omega, np.zeros(n ** d))
    k_gpu = pb.kernel_table().cpu().numpy()
    k_ref = kernel_table(n, d, omega).transpose(tuple(range(d))[::-1]).reshape(-1)
    err = np.abs(k_gpu - k_ref)
    assert err.max() <= 1e-13 * np.abs(k_ref).max()
    assert np.max(err / np.abs(k_ref)) <= 1e-13


@pytest.mark.parametrize("n,d", [(32, 2), (48, 2), (64, 2), (12, 3), (16, 3)])
def test_K_matvec_fp64(n, d):
    """FFT convolution (Stockham, radix 8/4/2/3) vs direct O(N^2) summation:
    relative L2 error <= 1e-12 (FP64 FFT error ~ eps log2(L^d))."""
    omega = 2 * np.pi * n / 8
    lsp, torch, plan, pb = _problem(n, d, omega, np.zeros(n ** d), max_nrhs=3)
    v = synth.random_complex((3, n ** d), seed=n + d)
    y = pb.apply_K(v).cpu().numpy()
    y_ref = apply_K_direct(v, n, d, omega)
    assert _rel(y, y_ref) <= 1e-12


@pytest.mark.parametrize("n,d", [(64, 2), (16, 3)])
def test_K_matvec_mixed(n, d):
    """complex64 convolution: relative L2 error <= 2e-6 (FP32 eps ~ 6e-8 times log2 L^d)."""
    omega = 2 * np.pi * n / 8
    lsp, torch, plan, pb = _problem(n, d, omega, np.zeros(n ** d), max_nrhs=2)
    v = synth.random_complex((2, n ** d), seed=7)
    y = pb.apply_K(v, precision=lsp.LSP_MIXED).cpu().numpy()
    y_ref = apply_K_direct(v, n, d, omega)
    assert _rel(y, y_ref) <= 2e-6


@pytest.mark.parametrize("key", ["c1"])
def test_operator_apply(key):
    """y = x + K(w^2 m x) vs the oracle operator, FP64, <= 1e-12."""
    w = synth.workload(key)
    n, d, omega, m = w["n"], w["d"], w["omega"], w["m"]
    lsp, torch, plan, pb = _problem(n, d, omega, m)
    x = synth.random_complex(n ** d, seed=3)
    y = pb.apply_op(x).cpu().numpy()[0]
    y_ref = Operator(n, d, omega, m).apply(x)
    assert _rel(y, y_ref) <= 1e-12


def _gpu_stencil_checks(pb, n, d, omega, tol_sig=1e-9, tol_alpha=1e-9):
    alpha, sigma, C = pb.stencils()
    kt = kernel_table(n, d, omega)
    sts = all_stencils(kt, d, n, b=2)
    for st in sts:
        sl = slot(st.offsets)
        a_gpu = alpha[st.c, sl]
        s = st.offsets.shape[0]
        # singular values, all of them, relative to their own size
        assert np.all(np.abs(sigma[st.c, :s] - st.sigma) <= tol_sig * st.sigma + 1e-15 * st.sigma[0])
        # same normalisation (unit norm, real positive centre)
        assert abs(abs(np.vdot(a_gpu, st.alpha)) - 1) <= 1e-12
        assert np.max(np.abs(a_gpu - st.alpha)) <= tol_alpha
        assert np.max(np.abs(C[st.c, sl] - st.C)) <= tol_alpha * np.max(np.abs(st.C))
        other = np.setdiff1d(np.arange(27), sl)
        assert np.all(alpha[st.c, other] == 0)
    return sts


@pytest.mark.parametrize("n,d", [(32, 2), (64, 2), (12, 3)])
def test_stencils(n, d):
    """Two-pass Gram + Jacobi null vectors vs dense SVD: every singular value to
    1e-9 relative, alpha and C entrywise to 1e-9 (same phase convention)."""
    omega = 2 * np.pi * n / 8
    lsp, torch, plan, pb = _problem(n, d, omega, np.zeros(n ** d))
    _gpu_stencil_checks(pb, n, d, omega)


@pytest.mark.parametrize("n,d", [(32, 2), (12, 3)])
def test_Q_and_M(n, d):
    """Q apply and the assembled M = [A + C w^2 m; B] vs the oracle's sparse matrices."""
    omega = 2 * np.pi * n / 8
    m = synth.medium_single_bump(n, d, 0.2, 0.15)
    lsp, torch, plan, pb = _problem(n, d, omega, m, max_nrhs=2)
    sts = all_stencils(kernel_table(n, d, omega), d, n, b=2)
    Q, M = build_QM(n, d, omega, m, sts)
    x = synth.random_complex((2, n ** d), seed=5)
    y = pb.apply_Q(x).cpu().numpy()
    assert _rel(y, (Q @ x.T).T) <= 1e-12
    Mv = pb.matrix().cpu().numpy()            # [N][3^d]
    Md = M.toarray()
    I = np.stack([(np.arange(n ** d) // n ** a) % n for a in range(d)], axis=1)
    for i in range(0, n ** d, max(1, n ** d // 97)):
        for q in range(3 ** d):
            o = np.array([(q // 3 ** a) % 3 - 1 for a in range(d)])
            j = I[i] + o
            if np.all((j >= 0) & (j < n)):
                jl = int(np.sum(j * n ** np.arange(d)))
                assert abs(Mv[i, q] - Md[i, jl]) <= 1e-12 * np.abs(Md).max()
            else:
                assert Mv[i, q] == 0


@pytest.mark.parametrize("n,d,prec,tol,dense", [(32, 2, "fp64", 1e-10, 1), (64, 2, "fp64", 1e-10, 1),
                                                (12, 3, "fp64", 1e-10, 1), (64, 2, "mixed", 1e-4, 1),
                                                (256, 2, "fp64", 1e-10, 1), (256, 2, "mixed", 1e-4, 1),
                                                (256, 2, "fp64", 1e-10, 0), (256, 2, "mixed", 1e-4, 0)])
def test_solve_M_vs_superlu(n, d, prec, tol, dense):
    """Multifrontal LU + triangular solves vs SuperLU: M^{-1} z, FP64 to 1e-10
    relative (kappa(M)-scaled rounding), complex64 fronts to 1e-4.  n = 256
    covers the one-wave diagonal-block factorisation (levels of 1024 fronts),
    the lookahead factorisation inside the trailing updates of the upper
    levels, and either the formed dense operators of the top five levels
    (dense = 1) or, on every level, the panel chains, with 512-thread
    workgroups on the wide levels (dense = 0)."""
    omega = 2 * np.pi * n / 8
    m = synth.medium_single_bump(n, d, 0.25, 0.12)
    lsp, torch, plan, pb = _problem(n, d, omega, m, max_nrhs=2, precision=prec, dense_sweeps=dense)
    assert (plan.stats()["dense_levels"] > 0) == bool(dense)
    pb.factor()
    sts = all_stencils(kernel_table(n, d, omega), d, n, b=2)
    Q, M = build_QM(n, d, omega, m, sts)
    P = Preconditioner(Q, M)
    z = synth.random_complex((2, n ** d), seed=9)
    x = pb.solve_M(z).cpu().numpy()
    x_ref = np.stack([P.solve_M(z[r]) for r in range(2)])
    assert _rel(x, x_ref) <= tol
    v = pb.apply_precond(z).cpu().numpy()
    v_ref = np.stack([P(z[r]) for r in range(2)])
    assert _rel(v, v_ref) <= tol


def test_c1_end_to_end_fp64():
    """2D n=32 workload: GPU FP64 GMRES vs the oracle: solution to 1e-8
    relative, iteration count within 1, true residual <= 1e-8."""
    w = synth.workload("c1")
    n, d, omega, m = w["n"], w["d"], w["omega"], w["m"]
    lsp, torch, plan, pb = _problem(n, d, omega, m)
    pb.factor()
    u, info, st = pb.solve(w["uI"])
    assert st == 0 and info[0]["converged"] and info[0]["relres_true"] <= 1e-8
    ref = OracleProblem(n, d, omega, m).solve(w["uI"][0])
    assert _rel(u.cpu().numpy()[0], ref.x) <= 1e-8
    assert abs(info[0]["iters"] - ref.iters) <= 1
    # the dense direct solve of the discrete system
    K = dense_K(n, d, omega)
    A = np.eye(n ** d) + K * (omega ** 2 * m)[None, :]
    u_star = np.linalg.solve(A, K @ (-omega ** 2 * m * w["uI"][0]))
    assert _rel(u.cpu().numpy()[0], u_star) <= np.linalg.cond(A) * 1e-8


def test_c1_end_to_end_mixed():
    """Mixed path (complex64 preconditioner and Arnoldi operator, complex128
    Arnoldi/residual/update): true residual <= 1e-8 (hard), and the error to
    the oracle solution is bounded by cond(A) * 1e-8."""
    w = synth.workload("c1")
    n, d, omega, m = w["n"], w["d"], w["omega"], w["m"]
    lsp, torch, plan, pb = _problem(n, d, omega, m, precision="mixed")
    pb.factor()
    u, info, st = pb.solve(w["uI"])
    assert st == 0 and info[0]["converged"] and info[0]["relres_true"] <= 1e-8
    ref = OracleProblem(n, d, omega, m).solve(w["uI"][0], tol=1e-12)
    assert _rel(u.cpu().numpy()[0], ref.x) <= 1e-7
    op = Operator(n, d, omega, m)
    g = op.rhs(w["uI"][0])
    assert np.linalg.norm(g - op.apply(u.cpu().numpy()[0])) <= 1e-8 * np.linalg.norm(g)


@pytest.mark.parametrize("n,d,prec,tol", [(128, 2, "fp64", 1e-12), (128, 2, "mixed", 2e-5),
                                          (16, 3, "fp64", 1e-12), (16, 3, "mixed", 2e-5)])
def test_dense_sweeps_match_panel_chains(n, d, prec, tol):
    """The dense levels' formed operators applied as matrix-vector products
    give the panel chains' M^{-1} z up to rounding: FP64 to 1e-12, complex64
    to 2e-5 (both sides round a complex64 chain of the same factor); three
    right-hand sides, so the sweeps run a group of two and a ragged one.  In
    3D (n = 16) the dense levels are the top four, fronts of up to 384 rows."""
    omega = 2 * np.pi * n / 8
    m = synth.medium_single_bump(n, d, 0.25, 0.12)
    z = synth.random_complex((3, n ** d), seed=31)
    out = []
    for dense in (1, 0):
        lsp, torch, plan, pb = _problem(n, d, omega, m, max_nrhs=3, precision=prec, dense_sweeps=dense)
        assert (plan.stats()["dense_levels"] > 0) == bool(dense)
        pb.factor()
        out.append(pb.solve_M(z).cpu().numpy())
    assert _rel(out[0], out[1]) <= tol


def test_dense_formation_lifecycle():
    """The dense levels' operators are formed on the library's side stream
    after lsp_factor returns: destroying a problem right after its
    factorisation, and factoring a problem twice before solving, leave
    every later solve bit-identical to a plain factor-then-solve."""
    n, d = 64, 2
    omega = 2 * np.pi * n / 8
    m = synth.medium_single_bump(n, d, 0.25, 0.12)
    z = synth.random_complex((1, n ** d), seed=41)
    lsp, torch, plan, pb = _problem(n, d, omega, m, precision="mixed")
    assert plan.stats()["dense_levels"] > 0
    pb.factor()
    ref = pb.solve_M(z).cpu().numpy()
    other = lsp.Problem(plan, omega, m)
    other.factor()
    del other  # destroyed while its formation may still run
    pb2 = lsp.Problem(plan, omega, m)
    pb2.factor()
    pb2.factor()  # the second factorisation waits for the first one's formation
    x = pb2.solve_M(z).cpu().numpy()
    assert np.array_equal(x, ref)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batched_equals_solo_bitwise(prec):
    """Lockstep batching: each right-hand side of a block of 5 (groups of 4 + 1
    in the panel-chain sweeps) is bit-identical to its solo solve.  The
    small-front levels run the matrix-core chains in both (16-column
    products, the unused columns zero), the middle levels the panel chains
    with groups of 4 and 1, the top levels the formed dense operators."""
    n, d = 48, 2
    omega = 2 * np.pi * n / 8
    rng = np.random.default_rng([14084495, 77])
    m = synth.medium_bumps(n, d, rng, 4, 0.2, 0.8, 0.05, 0.1, 0.0, 0.3)
    uI = synth.plane_waves(n, d, omega, synth.directions_2d(5, 0.3))
    lsp, torch, plan, pb = _problem(n, d, omega, m, max_nrhs=5, precision=prec)
    pb.factor()
    u_all, info_all, st = pb.solve(uI)
    assert st == 0
    for r in (0, 3, 4):
        u1, info1, st1 = pb.solve(uI[r:r + 1])
        assert st1 == 0
        assert torch.equal(u1[0], u_all[r])
        assert info1[0]["iters"] == info_all[r]["iters"]


def test_c2_full_size_fp64_and_mixed():
    """2D n=256 workload (the benchmark's): both paths reach a true residual
    <= 1e-8 as measured by the oracle's own FFT operator; FP64 matches the
    oracle's solution to 1e-8 with iterations within 1; mixed differs from it
    by at most cond-scaled 1e-7."""
    w = synth.workload("c2")
    n, d, omega, m = w["n"], w["d"], w["omega"], w["m"]
    ref = OracleProblem(n, d, omega, m).solve(w["uI"][0])
    op = Operator(n, d, omega, m)
    g = op.rhs(w["uI"][0])
    for prec in ("fp64", "mixed"):
        lsp, torch, plan, pb = _problem(n, d, omega, m, precision=prec)
        pb.factor()
        u, info, st = pb.solve(w["uI"])
        assert st == 0 and info[0]["converged"]
        u = u.cpu().numpy()[0]
        assert np.linalg.norm(g - op.apply(u)) <= 1e-8 * np.linalg.norm(g)
        if prec == "fp64":
            assert _rel(u, ref.x) <= 1e-8
            assert abs(info[0]["iters"] - ref.iters) <= 1
        else:
            assert _rel(u, ref.x) <= 1e-6


@pytest.mark.parametrize("n", [16, 24])
def test_3d_end_to_end(n):
    """3D Gaussian-bump medium, 2 directions: FP64 GPU vs oracle (1e-8,
    iterations within 1); n=24 uses FFT length 48 = 2^4 3 (radix 3)."""
    d = 3
    omega = 2 * np.pi * n / 8
    rng = np.random.default_rng([14084495, 3, n])
    m = synth.medium_bumps(n, d, rng, 3, 0.3, 0.7, 0.08, 0.12, 0.0, 0.3)
    uI = synth.plane_waves(n, d, omega, synth.directions_fibonacci(2, rng))
    lsp, torch, plan, pb = _problem(n, d, omega, m, max_nrhs=2)
    pb.factor()
    u, info, st = pb.solve(uI)
    assert st == 0
    prob = OracleProblem(n, d, omega, m)
    for r in range(2):
        ref = prob.solve(uI[r])
        assert _rel(u.cpu().numpy()[r], ref.x) <= 1e-8
        assert abs(info[r]["iters"] - ref.iters) <= 1


def test_kernel_timing_registry():
    """Per-kernel HIP-event timing records the library's launches by name."""
    lsp, torch = _lsp()
    w = synth.workload("c1")
    lsp.timing_reset()
    lsp.timing_enable(True)
    try:
        plan = lsp.Plan(w["n"], w["d"])
        pb = lsp.Problem(plan, w["omega"], w["m"])
        pb.factor()
        pb.solve(w["uI"])
    finally:
        lsp.timing_enable(False)
    t = lsp.timing_read()
    names = {k.split(" ")[0] for k in t}
    assert {"ktable", "gram", "eigen", "diag_lu", "gemm_update", "fwd", "bwd", "fft_conv"} <= names
    assert all(ms > 0 and cnt > 0 for ms, cnt in t.values())


def test_tile_tables_give_same_factor():
    """Every trailing-update tile shape (32/64/128) yields the same M^{-1} z up
    to rounding (1e-12), and the autotuner returns a valid per-level table."""
    n, d = 64, 2
    omega = 2 * np.pi * n / 8
    m = synth.medium_single_bump(n, d, 0.25, 0.12)
    lsp, torch, plan, pb = _problem(n, d, omega, m)
    nl = plan.stats()["nlevels"]
    z = synth.random_complex((1, n ** d), seed=21)
    ref = None
    for t in (32, 64, 128):
        plan.set_tiles([t] * nl)
        pb.factor()
        x = pb.solve_M(z).cpu().numpy()
        if ref is None:
            ref = x
        assert _rel(x, ref) <= 1e-12
    from paper_1408_4495_amd.autotune import tune_tiles
    res = tune_tiles(48, 2, "fp64", reps=1)
    assert len(res["tiles"]) > 0 and all(t in (32, 64, 128) for t in res["tiles"])
    assert res["factor_ms"] <= min(res["uniform_ms"].values()) * 1.05


@pytest.mark.parametrize("n,d,prec,tol", [(32, 3, "fp64", 1e-12), (32, 3, "mixed", 2e-5),
                                          (48, 3, "mixed", 2e-5)])
def test_blocked_sweeps_match_panel_chains(n, d, prec, tol):
    """Blocked sweeps (a panel chain per 256-row super-block and wide
    matrix-vector products; 3D n = 32: the top three levels, fronts of up to
    1536 rows, the root level two super-blocks; n = 48: six levels, up to
    nine super-blocks) give the panel chains' M^{-1} z up to rounding: FP64
    to 1e-12, complex64 to 2e-5.  Three right-hand sides: a chain group of
    two and a ragged one in the panel-chain path."""
    omega = 2 * np.pi * n / 8
    m = synth.medium_single_bump(n, d, 0.25, 0.12)
    z = synth.random_complex((3, n ** d), seed=37)
    out = []
    for blocked in (1, 0):
        lsp, torch, plan, pb = _problem(n, d, omega, m, max_nrhs=3, precision=prec, blocked_sweeps=blocked)
        pb.factor()
        out.append(pb.solve_M(z).cpu().numpy())
        del pb
    assert _rel(out[0], out[1]) <= tol


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_blocked_batched_equals_solo_bitwise(prec):
    """On blocked levels each right-hand side of a block of 17 (a 16-wide and
    a ragged matrix-vector group, chain groups of 8, 8 and 1) gets its solo
    M^{-1} z bit for bit."""
    n, d = 32, 3
    omega = 2 * np.pi * n / 8
    m = synth.medium_single_bump(n, d, 0.25, 0.12)
    z = synth.random_complex((17, n ** d), seed=43)
    lsp, torch, plan, pb = _problem(n, d, omega, m, max_nrhs=17, precision=prec)
    pb.factor()
    x_all = pb.solve_M(z)
    for r in (0, 9, 16):
        x1 = pb.solve_M(z[r:r + 1])
        assert torch.equal(x1[0], x_all[r])


@pytest.mark.parametrize("n,d,prec,tol", [(128, 2, "fp64", 1e-12), (128, 2, "mixed", 2e-5),
                                          (16, 3, "fp64", 1e-12), (16, 3, "mixed", 2e-5)])
def test_mchain_levels_match_panel_chains(n, d, prec, tol):
    """Small-front levels swept by panel chains on the matrix cores (plans
    for blocks of right-hand sides: 2D n = 128 its six lowest levels, 3D
    n = 16 its two lowest) give the vector panel chains' M^{-1} z up to
    rounding (FP64 1e-12, complex64 2e-5); 5 right-hand sides."""
    omega = 2 * np.pi * n / 8
    m = synth.medium_single_bump(n, d, 0.25, 0.12)
    z = synth.random_complex((5, n ** d), seed=53)
    out = []
    for dense in (1, 0):
        lsp, torch, plan, pb = _problem(n, d, omega, m, max_nrhs=5, precision=prec, dense_sweeps=dense)
        assert (plan.stats()["mchain_levels"] > 0) == bool(dense)
        pb.factor()
        out.append(pb.solve_M(z).cpu().numpy())
        del pb
    assert _rel(out[0], out[1]) <= tol
