"""Problems set up and factored at the same time on four streams (four host
threads, as the request loop runs them) give stencils (Section 3.1: alpha,
sigma, C of every class) and preconditioner applications M^{-1} z bit for bit
equal to the same problems run one at a time.  A workgroup-level race in a
set-up or factor kernel shows here as a mismatch: the kernels' wave
interleaving changes when other work shares the compute units."""
import threading

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def test_concurrent_setup_and_factor_match_solo():
    import torch
    from paper_1408_4495_amd import lsp
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lsp.load()
    specs = synth.serving_requests(24, 1.0, seed=5, sizes=[(32, 3), (48, 3), (128, 2)])
    plans = {}
    for s in specs:
        if (s["n"], s["d"]) not in plans:
            plans[(s["n"], s["d"])] = lsp.Plan(s["n"], s["d"], max_nrhs=1, precision="mixed")
    rng = np.random.default_rng([2025, 11])
    zs = {k: rng.standard_normal(k[0] ** k[1]) + 1j * rng.standard_normal(k[0] ** k[1]) for k in plans}
    streams = [torch.cuda.Stream() for _ in range(4)]

    def probe(s, stream):
        with torch.cuda.stream(stream):
            key = (s["n"], s["d"])
            m = torch.tensor(s["m"], dtype=torch.float64, device="cuda:0")
            pb = lsp.Problem(plans[key], s["omega"], m, stream=stream)
            al, sg, C = pb.stencils()
            pb.factor()
            x = pb.solve_M(zs[key]).cpu().numpy()
            stream.synchronize()
            del pb
            return al, sg, C, x

    print("[concurrency] solo runs", flush=True)
    solo = [probe(s, streams[0]) for s in specs]
    for rep in range(3):
        print(f"[concurrency] concurrent pass {rep}", flush=True)
        res = [None] * len(specs)
        errs = []
        lock = threading.Lock()
        nxt = [0]

        def worker(w):
            while True:
                with lock:
                    i = nxt[0]
                    nxt[0] += 1
                if i >= len(specs):
                    return
                try:
                    res[i] = probe(specs[i], streams[w])
                except Exception as e:  # reported below
                    errs.append((i, repr(e)))

        th = [threading.Thread(target=worker, args=(w,)) for w in range(4)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        assert not errs, f"pass {rep}: {errs}"
        for i, s in enumerate(specs):
            for j, name in enumerate(("alpha", "sigma", "C", "M^-1 z")):
                assert np.array_equal(solo[i][j], res[i][j]), \
                    f"pass {rep}, problem {i} (n={s['n']}, d={s['d']}): {name} differs from the solo run"
