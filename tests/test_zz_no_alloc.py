"""The allocation-free operator entry point (static per-device scratch)
against lsp_apply_op on the same inputs: equal bit for bit (same kernels,
same arithmetic), on two calls in a row, the second with a smaller input,
in both precisions; sizes beyond the scratch are refused."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _lsp():
    import torch
    from paper_1408_4495_amd import lsp
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lsp.load()
    return lsp, torch


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_equals_workspace_entry_point(prec):
    lsp, torch = _lsp()
    code = lsp.LSP_MIXED if prec == "mixed" else lsp.LSP_FP64
    cases = [(64, 2, 3), (32, 2, 1), (16, 3, 2)]   # second call smaller than the first
    for n, d, nrhs in cases:
        omega = 2 * np.pi * n / 8
        m = synth.medium_single_bump(n, d, 0.25, 0.12)
        plan = lsp.Plan(n, d, max_nrhs=nrhs, precision=prec)
        pb = lsp.Problem(plan, omega, m)
        x = synth.random_complex((nrhs, n ** d), seed=n + nrhs)
        y_ws = pb.apply_op(x, precision=code)
        y_na = pb.apply_op_noalloc(x, precision=code)
        torch.cuda.synchronize()
        assert torch.equal(y_na, y_ws), (n, d, nrhs)
        # and a repeat on the same problem after another problem used the scratch
        assert torch.equal(pb.apply_op_noalloc(x, precision=code), y_ws)


def test_noalloc_refuses_oversize():
    lsp, torch = _lsp()
    n, d = 512, 2            # (2n)^2 complex128 = 16 MiB per right-hand side
    plan = lsp.Plan(n, d, max_nrhs=3)
    pb = lsp.Problem(plan, 2 * np.pi * n / 8, np.zeros(n * n))
    x = torch.zeros((3, n * n), dtype=torch.complex128, device="cuda:0")
    with pytest.raises(lsp.LspError) as e:
        pb.apply_op_noalloc(x)
    assert e.value.status == 1 and "static scratch" in str(e.value)
    # two right-hand sides fit exactly
    y = pb.apply_op_noalloc(x[:2])
    torch.cuda.synchronize()
    assert torch.count_nonzero(y) == 0
