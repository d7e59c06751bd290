"""Serving loop: requests of different n, d, w and media admitted by HBM
footprint, overlapping on per-slot streams; each result must equal the
request's solo run (bit-for-bit: every kernel is deterministic and
independent of concurrent work)."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _requests(seed, arrival_gap):
    rng = np.random.default_rng([14084495, 4, seed])
    sizes = [(32, 2), (48, 2), (64, 2), (12, 3), (16, 3), (32, 2)]
    out = []
    from paper_1408_4495_amd.serve import Request
    for k, (n, d) in enumerate(sizes):
        p = synth.media.request_problem(n, d, 1 + (k % 3), rng)
        out.append(Request(k, n, d, p["omega"], p["m"], p["uI"], arrival=k * arrival_gap))
    return out


def test_mix_equals_solo_and_overlaps():
    import torch
    from paper_1408_4495_amd.serve import Server
    srv = Server(precision="mixed", slots=3)
    mix = _requests(1, 0.0)
    rep = srv.run(mix)
    assert rep["all_converged"] and rep["requests"] == len(mix)
    assert rep["peak_concurrency"] >= 2
    assert rep["latency_ms"]["p99"] >= rep["latency_ms"]["p50"] > 0
    solo_srv = Server(precision="mixed", slots=1)
    for r in mix:
        alone = _requests(1, 0.0)[r.id]
        solo_srv.run([alone])
        assert np.array_equal(alone.u, r.u), f"request {r.id} differs between mix and solo"
        assert [x["iters"] for x in alone.info] == [x["iters"] for x in r.info]
        assert all(x["relres_true"] <= 1e-8 for x in r.info)
    torch.cuda.synchronize()


def test_admission_by_footprint():
    """Requests are admitted only while their summed footprint fits the budget:
    three equal-size requests under a budget of one footprint run one at a
    time; a request above the budget is refused."""
    from paper_1408_4495_amd.serve import Server, Request
    rng = np.random.default_rng([14084495, 4, 2])
    reqs = []
    for k in range(3):
        p = synth.media.request_problem(48, 2, 2, rng)
        reqs.append(Request(k, 48, 2, p["omega"], p["m"], p["uI"], arrival=0.0))
    probe = Server(precision="mixed", slots=3)
    fp = probe.footprint(reqs[0])
    assert all(probe.footprint(r) == fp for r in reqs)
    tight = Server(precision="mixed", slots=3, hbm_budget=fp)
    rep = tight.run(reqs)
    assert rep["all_converged"] and rep["peak_concurrency"] == 1
    assert rep["peak_admitted_bytes"] <= fp
    roomy = Server(precision="mixed", slots=3, hbm_budget=3 * fp)
    rep = roomy.run(reqs)
    assert rep["peak_admitted_bytes"] <= 3 * fp
    too_small = Server(precision="mixed", slots=3, hbm_budget=fp // 4)
    with pytest.raises(ValueError):
        too_small.run(reqs)
