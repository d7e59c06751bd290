"""The result of set-up, factorisation and solve does not depend on what the
caller's workspaces held before: the problem and solve workspaces are filled
with zero bytes, with 0xFF (a NaN in every floating-point format) and with
0x7F (huge finite values) before set-up, and the solutions must agree bit for
bit.  A kernel that reads a workspace entry before writing it, or multiplies
a stale entry by zero, fails here."""
import ctypes

import numpy as np
import pytest

import synth
from synth.media import request_problem

pytestmark = pytest.mark.gpu


def _run(lsp, torch, plan, omega, m_t, uI_t, fill):
    stream = torch.cuda.current_stream()
    nrhs = uI_t.shape[0]
    pbytes, _ = plan.bytes(1)
    _, sbytes = plan.bytes(nrhs)
    ws = torch.full((pbytes,), fill, dtype=torch.uint8, device="cuda:0")
    h = ctypes.c_void_p()
    lsp._check(lsp._lib.lsp_setup(plan._h, float(omega), lsp._ptr(m_t), lsp._ptr(ws), pbytes,
                                  ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
    # the binding's problem object around the raw handle and the filled workspaces
    pb = object.__new__(lsp.Problem)
    pb.torch, pb.plan, pb.device, pb.stream = torch, plan, torch.device("cuda:0"), stream
    pb.ws, pb._h, pb.omega, pb.N, pb._phases = ws, h, float(omega), plan.n ** plan.d, {}
    pb._solve_ws = torch.full((sbytes,), fill, dtype=torch.uint8, device="cuda:0")
    pb.factor()
    u, info, st = pb.solve(uI_t)
    torch.cuda.synchronize()
    out = torch.view_as_real(u).cpu().numpy().copy()
    iters = [x["iters"] for x in info]
    del pb
    return out, iters, st


@pytest.mark.parametrize("n,d,nrhs,prec", [(32, 3, 21, "mixed"), (48, 3, 8, "mixed"), (32, 3, 4, "fp64"),
                                           (128, 2, 8, "mixed"), (256, 2, 4, "fp64")])
def test_result_independent_of_workspace_contents(n, d, nrhs, prec):
    import torch
    from paper_1408_4495_amd import lsp
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lsp.load()
    rng = np.random.default_rng([2024, n, d, nrhs])
    prob = request_problem(n, d, nrhs, rng)
    plan = lsp.Plan(n, d, max_nrhs=max(nrhs, 1), precision=prec)
    m_t = torch.tensor(prob["m"], dtype=torch.float64, device="cuda:0")
    uI_t = torch.tensor(prob["uI"], dtype=torch.complex128, device="cuda:0")
    ref = None
    for fill in (0x00, 0xFF, 0x7F):
        print(f"[ws-init] n={n} d={d} nrhs={nrhs} {prec} fill=0x{fill:02X}", flush=True)
        u, iters, st = _run(lsp, torch, plan, prob["omega"], m_t, uI_t, fill)
        assert st == 0, f"fill 0x{fill:02X}: status {st}"
        assert np.all(np.isfinite(u)), f"fill 0x{fill:02X}: non-finite solution"
        if ref is None:
            ref = (u, iters)
        else:
            assert iters == ref[1], f"fill 0x{fill:02X}: iterations {iters} vs {ref[1]}"
            bad = np.argwhere(u != ref[0])
            assert bad.size == 0, f"fill 0x{fill:02X}: {len(bad)} entries differ, first at {bad[:4].tolist()}"
