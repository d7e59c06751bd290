"""Options and failure paths of the C ABI on the GPU, each against the oracle:
the buffer constant b of Section 3.1 other than the default, GMRES with a
short restart and with an iteration cap (LSP_ERR_NOCONV, Section 3.3
experiments' solver), the stencil application Q v (eq:PC) in isolation (and its
row blocks, batched against solo bit for bit), the
complex64 factor in 3D, and a medium carrying a NaN (LSP_ERR_SINGULAR)."""
import numpy as np
import pytest

import synth
from oracle.greens import kernel_table
from oracle.stencil import all_stencils, StencilClass, class_offsets
from oracle.sparse import build_QM, Preconditioner
from oracle.solve import OracleProblem
from oracle.gmres import gmres

pytestmark = pytest.mark.gpu


def _lsp():
    import torch
    from paper_1408_4495_amd import lsp
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lsp.load()
    return lsp, torch


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


def _slots(st):
    return np.sum((st.offsets + 1) * (3 ** np.arange(st.offsets.shape[1])), axis=1)


@pytest.mark.parametrize("n,d,b", [(32, 2, 1), (32, 2, 4), (12, 3, 1), (12, 3, 4)])
def test_buffer_b_stencils_and_matrix(n, d, b):
    """Boundary far sets with b = 1 and 4 (Section 3.1): every singular value
    to 1e-9 relative, alpha and C entrywise 1e-9, M's entries 1e-12 of max."""
    lsp, torch = _lsp()
    omega = 2 * np.pi * n / 8
    m = synth.medium_single_bump(n, d, 0.2, 0.15)
    plan = lsp.Plan(n, d, buffer_b=b)
    pb = lsp.Problem(plan, omega, m)
    alpha, sigma, C = pb.stencils()
    sts = all_stencils(kernel_table(n, d, omega), d, n, b)
    for st in sts:
        sl = _slots(st)
        s = st.offsets.shape[0]
        assert np.all(np.abs(sigma[st.c, :s] - st.sigma) <= 1e-9 * st.sigma + 1e-15 * st.sigma[0])
        assert np.max(np.abs(alpha[st.c, sl] - st.alpha)) <= 1e-9
        assert np.max(np.abs(C[st.c, sl] - st.C)) <= 1e-9 * np.max(np.abs(st.C))
    _, M = build_QM(n, d, omega, m, sts)
    Mv = pb.matrix().cpu().numpy()
    Md = M.toarray()
    I = np.stack([(np.arange(n ** d) // n ** a) % n for a in range(d)], axis=1)
    for i in range(0, n ** d, max(1, n ** d // 89)):
        for q in range(3 ** d):
            o = np.array([(q // 3 ** a) % 3 - 1 for a in range(d)])
            j = I[i] + o
            if np.all((j >= 0) & (j < n)):
                jl = int(np.sum(j * n ** np.arange(d)))
                assert abs(Mv[i, q] - Md[i, jl]) <= 1e-12 * np.abs(Md).max()


@pytest.mark.parametrize("b", [1, 4])
def test_buffer_b_end_to_end(b):
    """2D n = 32 workload solved with b = 1 and 4: FP64 solution within 1e-8
    of the oracle's (same b), iterations within 1."""
    lsp, torch = _lsp()
    w = synth.workload("c1")
    n, d, omega, m = w["n"], w["d"], w["omega"], w["m"]
    plan = lsp.Plan(n, d, buffer_b=b)
    pb = lsp.Problem(plan, omega, m)
    pb.factor()
    u, info, st = pb.solve(w["uI"])
    assert st == 0 and info[0]["converged"]
    ref = OracleProblem(n, d, omega, m, b=b).solve(w["uI"][0])
    assert _rel(u.cpu().numpy()[0], ref.x) <= 1e-8
    assert abs(info[0]["iters"] - ref.iters) <= 1


def test_restart_two_fp64():
    """GMRES(2) on the 2D n = 32 workload (restarts after every second
    Arnoldi step): FP64 solution within 1e-8 of the oracle's GMRES(2),
    iteration counts equal."""
    lsp, torch = _lsp()
    w = synth.workload("c1")
    n, d, omega, m = w["n"], w["d"], w["omega"], w["m"]
    plan = lsp.Plan(n, d, restart=2)
    pb = lsp.Problem(plan, omega, m)
    pb.factor()
    u, info, st = pb.solve(w["uI"])
    assert st == 0 and info[0]["converged"]
    ref = OracleProblem(n, d, omega, m).solve(w["uI"][0], restart=2)
    assert ref.converged and ref.iters > 2
    assert _rel(u.cpu().numpy()[0], ref.x) <= 1e-8
    assert info[0]["iters"] == ref.iters


def test_max_iters_noconv():
    """max_iters = 1: the solve returns LSP_ERR_NOCONV with the information
    filled, and u is the one-step iterate, the oracle's to 1e-8."""
    lsp, torch = _lsp()
    w = synth.workload("c1")
    n, d, omega, m = w["n"], w["d"], w["omega"], w["m"]
    plan = lsp.Plan(n, d, max_iters=1)
    pb = lsp.Problem(plan, omega, m)
    pb.factor()
    u, info, st = pb.solve(w["uI"])
    assert st == 6
    assert info[0]["iters"] == 1 and not info[0]["converged"]
    ref = OracleProblem(n, d, omega, m).solve(w["uI"][0], max_iters=1)
    assert not ref.converged and ref.iters == 1
    assert _rel(u.cpu().numpy()[0], ref.x) <= 1e-8
    assert abs(info[0]["relres_true"] - ref.relres) <= 1e-6 * ref.relres
    assert info[0]["t_solve"] > 0 and info[0]["t_factor"] > 0 and info[0]["t_setup"] > 0


@pytest.mark.parametrize("n,d", [(32, 2), (12, 3)])
def test_Q_apply_exact(n, d):
    """z = Q v alone: the GPU's stencil application against the oracle's
    sparse Q assembled from the GPU's own stencil coefficients (so the
    stencils' rounding is common to both): relative L2 error <= 1e-14."""
    lsp, torch = _lsp()
    omega = 2 * np.pi * n / 8
    plan = lsp.Plan(n, d, max_nrhs=2)
    pb = lsp.Problem(plan, omega, np.zeros(n ** d))
    alpha, sigma, C = pb.stencils()
    sts = []
    for c in range(3 ** d):
        off = class_offsets(c, d)
        sl = np.sum((off + 1) * (3 ** np.arange(d)), axis=1)
        sts.append(StencilClass(c, off, alpha[c, sl], sigma[c, :off.shape[0]], C[c, sl]))
    Q, _ = build_QM(n, d, omega, np.zeros(n ** d), sts)
    x = synth.random_complex((2, n ** d), seed=61)
    y = pb.apply_Q(x).cpu().numpy()
    y_ref = (Q @ x.T).T
    assert _rel(y, y_ref) <= 1e-14


def test_Q_apply_row_blocks_bitwise():
    """2D n = 256: the stencil product's row blocks shrink with the number of
    right-hand sides (16 right-hand sides: 2 rows per workgroup, one: 1), yet
    each point's sum is the same, so a batched product equals the solo ones
    bit for bit; and it matches the oracle's Q built from the GPU's stencils
    (relative 1e-14)."""
    lsp, torch = _lsp()
    n, d = 256, 2
    omega = 2 * np.pi * n / 8
    plan = lsp.Plan(n, d, max_nrhs=16)
    pb = lsp.Problem(plan, omega, np.zeros(n ** d))
    x = synth.random_complex((16, n ** d), seed=62)
    y = pb.apply_Q(x).cpu().numpy()
    for r in (0, 7, 15):
        assert np.array_equal(pb.apply_Q(x[r:r + 1]).cpu().numpy()[0], y[r])
    alpha, sigma, C = pb.stencils()
    sts = []
    for c in range(3 ** d):
        off = class_offsets(c, d)
        sl = np.sum((off + 1) * (3 ** np.arange(d)), axis=1)
        sts.append(StencilClass(c, off, alpha[c, sl], sigma[c, :off.shape[0]], C[c, sl]))
    Q, _ = build_QM(n, d, omega, np.zeros(n ** d), sts)
    assert _rel(y[:2], (Q @ x[:2].T).T) <= 1e-14


@pytest.mark.parametrize("n", [12, 16])
def test_solve_M_3d_complex64(n):
    """complex64 fronts and sweeps in 3D against SuperLU's FP64 M^{-1} z: 1e-4
    relative (single-precision factor of M)."""
    lsp, torch = _lsp()
    d = 3
    omega = 2 * np.pi * n / 8
    m = synth.medium_single_bump(n, d, 0.25, 0.12)
    plan = lsp.Plan(n, d, max_nrhs=2, precision="mixed")
    pb = lsp.Problem(plan, omega, m)
    pb.factor()
    sts = all_stencils(kernel_table(n, d, omega), d, n, b=2)
    Q, M = build_QM(n, d, omega, m, sts)
    P = Preconditioner(Q, M)
    z = synth.random_complex((2, n ** d), seed=67)
    x = pb.solve_M(z).cpu().numpy()
    x_ref = np.stack([P.solve_M(z[r]) for r in range(2)])
    assert _rel(x, x_ref) <= 1e-4


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_nan_medium_is_singular(prec):
    """A NaN in the medium reaches the fronts through M's interior rows; the
    factorisation reports LSP_ERR_SINGULAR and a solve is then refused with
    LSP_ERR_STATE.  Only NaN arithmetic, no faulting access."""
    lsp, torch = _lsp()
    n, d = 32, 2
    m = synth.medium_single_bump(n, d, 0.2, 0.1)
    m[n * (n // 2) + n // 2] = np.nan
    plan = lsp.Plan(n, d, precision=prec)
    pb = lsp.Problem(plan, 2 * np.pi * 4, m)
    with pytest.raises(lsp.LspError) as e:
        pb.factor()
    assert e.value.status == 5
    with pytest.raises(lsp.LspError) as e2:
        pb.solve(np.ones((1, n * n), dtype=np.complex128))
    assert e2.value.status == 4


@pytest.mark.parametrize("n,d", [(32, 2), (64, 3)])
def test_fitted_self_term(n, d):
    """self_term = 2 (the fourth-order one-point correction fitted to a
    Gaussian probe): the GPU's table (k_0 from the host) against the
    oracle's, k_0 to 2e-12 (lattice-sum rounding), the rest to 1e-13; and
    the 2D n = 32 workload solved with it against the oracle with the same
    self term (FP64, 1e-8, iterations within 1)."""
    lsp, torch = _lsp()
    omega = 2 * np.pi * n / 8
    plan = lsp.Plan(n, d, self_term=2)
    pb = lsp.Problem(plan, omega, np.zeros(n ** d))
    k = pb.kernel_table().cpu().numpy()
    ref = kernel_table(n, d, omega, self_term_mode=2).transpose(tuple(range(d))[::-1]).reshape(-1)
    assert abs(k[0] - ref[0]) <= 2e-12 * abs(ref[0])
    assert np.max(np.abs(k[1:] - ref[1:])) <= 1e-13 * np.abs(ref).max()
    if d == 2:
        w = synth.workload("c1")
        plan = lsp.Plan(w["n"], 2, self_term=2)
        pb = lsp.Problem(plan, w["omega"], w["m"])
        pb.factor()
        u, info, st = pb.solve(w["uI"])
        assert st == 0
        sol = OracleProblem(w["n"], 2, w["omega"], w["m"], self_term=2).solve(w["uI"][0])
        assert _rel(u.cpu().numpy()[0], sol.x) <= 1e-8
        assert abs(info[0]["iters"] - sol.iters) <= 1


@pytest.mark.parametrize("n,d", [(32, 2), (16, 3)])
def test_cell_self_term(n, d):
    """self_term = 1 (k_0 = the integral of G over the cell, Section 2.1's
    local correction): the GPU's k_0 (Gauss-Legendre over the cell's faces)
    against the oracle's Cartesian quadrature to 1e-11 relative, the rest of
    the table unchanged; and the 2D n = 32 workload solved with it against
    the oracle with the same self-term (FP64, 1e-8, iterations within 1)."""
    lsp, torch = _lsp()
    omega = 2 * np.pi * n / 8
    plan = lsp.Plan(n, d, self_term=1)
    pb = lsp.Problem(plan, omega, np.zeros(n ** d))
    k = pb.kernel_table().cpu().numpy()
    ref = kernel_table(n, d, omega, self_term_mode=1).transpose(tuple(range(d))[::-1]).reshape(-1)
    assert abs(k[0] - ref[0]) <= 1e-11 * abs(ref[0])
    assert np.max(np.abs(k[1:] - ref[1:])) <= 1e-13 * np.abs(ref).max()
    if d == 2:
        w = synth.workload("c1")
        plan = lsp.Plan(w["n"], 2, self_term=1)
        pb = lsp.Problem(plan, w["omega"], w["m"])
        pb.factor()
        u, info, st = pb.solve(w["uI"])
        assert st == 0
        sol = OracleProblem(w["n"], 2, w["omega"], w["m"], self_term=1).solve(w["uI"][0])
        assert _rel(u.cpu().numpy()[0], sol.x) <= 1e-8
        assert abs(info[0]["iters"] - sol.iters) <= 1
