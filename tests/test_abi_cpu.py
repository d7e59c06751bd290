"""Host-side checks of the C ABI (no GPU): the library loads, exports every
symbol include/lsp.h declares, validates arguments, and plans nested
dissection with the expected structure."""
import os
import re
import subprocess

import numpy as np
import pytest

import paper_1408_4495_amd as pkg
from paper_1408_4495_amd import lsp as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "lsp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lsp_[A-Za-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        from paper_1408_4495_amd import build
        build.build()
    return L.load()


def test_exports_every_declared_symbol(lib):
    declared = _declared()
    assert set(declared) == set(L.EXPORTED)
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (lsp_[A-Za-z_]+)\b", out))
    for name in declared:
        assert name in exported, name
        assert hasattr(lib, name)


def test_status_strings(lib):
    for code in range(7):
        assert lib.lsp_status_string(code)


@pytest.mark.parametrize("n,d,msg", [(3, 2, "n must"), (32, 4, "d must"), (5000, 2, "n must"),
                                     (14, 2, "factor")])
def test_plan_rejects_bad_shapes(lib, n, d, msg):
    with pytest.raises(L.LspError) as e:
        L.Plan(n, d)
    assert e.value.status == 1 and msg in str(e.value)


def test_plan_rejects_bad_options(lib):
    with pytest.raises(L.LspError):
        L.Plan(32, 2, restart=0)
    with pytest.raises(L.LspError):
        L.Plan(32, 2, restart=40)
    with pytest.raises(L.LspError):
        L.Plan(32, 2, buffer_b=31)
    with pytest.raises(L.LspError):
        L.Plan(32, 2, panel=64)
    with pytest.raises(L.LspError):
        L.Plan(32, 2, max_nrhs=0)


@pytest.mark.parametrize("n,d,fronts,maxf", [(32, 2, 31, 81), (256, 2, 2047, 385),
                                             (64, 3, 8191, 6144), (48, 3, 8191, 3456)])
def test_nested_dissection_structure(lib, n, d, fronts, maxf):
    """Geometric nested dissection with 1-wide separators: every grid point is
    eliminated once (the plan checks sum p = N and that each child's boundary
    lies in its parent front), and the tree matches the box recursion."""
    s = L.Plan(n, d).stats()
    assert s["N"] == n ** d and s["L"] == 2 * n
    assert s["nfronts"] == fronts and s["max_front"] == maxf
    assert s["max_pivots"] >= n ** (d - 1)      # the top separator is a full line / plane
    assert s["factor_flops"] > 0 and s["factor_entries"] <= s["front_entries"]


def test_plan_bytes_grow_with_rhs(lib):
    p = L.Plan(64, 2, max_nrhs=8)
    pb1, sb1 = p.bytes(1)
    pb8, sb8 = p.bytes(8)
    assert pb1 == pb8 and sb8 > 7 * sb1 * 0.9
    pm, _ = p.bytes(1, precision=L.LSP_MIXED)
    assert pm < pb1
    with pytest.raises(L.LspError):
        p.bytes(9)


def test_setup_rejects_bad_arguments_without_touching_gpu(lib):
    import ctypes
    p = L.Plan(16, 2)
    h = ctypes.c_void_p()
    # null medium / workspace and non-positive omega are rejected before any HIP call
    st = lib.lsp_setup(p._h, 5.0, None, None, 0, None, ctypes.byref(h))
    assert st == 1
    st = lib.lsp_setup(p._h, -1.0, ctypes.c_void_p(8), ctypes.c_void_p(8), 1 << 40, None, ctypes.byref(h))
    assert st == 1
    buf = ctypes.create_string_buffer(256)
    lib.lsp_last_error(buf, 256)
    assert b"omega" in buf.value
    assert lib.lsp_factor(None) == 1


def test_dense_sweep_levels(lib):
    """Dense sweep levels (at most 16 fronts, more than one panel, at most
    1024 rows): n = 8 in 2D is one front of 64 pivots and no boundary, so
    its operators hold 2 x 64^2 entries and no panel is left to the chains,
    whose reads would be two 32 x 32 inverse blocks and the 32 x 32 block
    below the first; at n = 256 the top five levels (16, 8, 4, 2, 1 fronts)
    are dense, and the problem's device memory grows by exactly the
    operators (2 entries per m p)."""
    q1, q0 = L.Plan(8, 2).stats(), L.Plan(8, 2, dense_sweeps=0).stats()
    assert q1["dense_levels"] == 1 and q1["dense_entries"] == 64 * 64 and q1["sweep_entries"] == 0
    assert q0["dense_levels"] == 0 and q0["dense_entries"] == 0 and q0["sweep_entries"] == 3 * 32 * 32
    p1, p0 = L.Plan(256, 2, blocked_sweeps=0), L.Plan(256, 2, dense_sweeps=0, blocked_sweeps=0)
    s1, s0 = p1.stats(), p0.stats()
    assert s1["dense_levels"] == 5 and s0["dense_levels"] == 0
    assert s1["sweep_entries"] < s0["sweep_entries"] and s1["dense_entries"] > 0
    for prec, esz in ((L.LSP_FP64, 16), (L.LSP_MIXED, 8)):
        grow = p1.bytes(1, prec)[0] - p0.bytes(1, prec)[0]
        assert 0 <= grow - 2 * s1["dense_entries"] * esz < 256


def test_blocked_sweep_levels(lib):
    """Blocked sweep levels: 3D n = 32 sweeps its three top non-dense levels
    (8, 4, 2 fronts of more than 1024 rows) blocked; each front keeps a
    forward and a backward 256 x 256 operator per 256-pivot super-block, so
    the problem's device memory grows by exactly 2 blocked_entries entries
    over the plan without blocked levels, and the solve workspace by the
    blocked sweeps' work buffers only."""
    b1, b0 = L.Plan(32, 3, max_nrhs=4), L.Plan(32, 3, max_nrhs=4, blocked_sweeps=0)
    s1, s0 = b1.stats(), b0.stats()
    assert s1["blocked_levels"] == 3 and s0["blocked_levels"] == 0
    assert s1["dense_levels"] == s0["dense_levels"]
    # fronts of those levels: 8 x 256, 4 x 256, 2 x 512 pivots -> 8 + 4 + 4 super-blocks
    assert s1["blocked_entries"] == 16 * 256 * 256
    for prec, esz in ((L.LSP_FP64, 16), (L.LSP_MIXED, 8)):
        grow = b1.bytes(4, prec)[0] - b0.bytes(4, prec)[0]
        assert 0 <= grow - 2 * s1["blocked_entries"] * esz < 256
        assert b1.bytes(4, prec)[1] > b0.bytes(4, prec)[1]
    # every non-dense, non-small level with blocked_sweeps = 2
    assert L.Plan(32, 3, blocked_sweeps=2).stats()["blocked_levels"] > s1["blocked_levels"]


def test_lookahead_schedule_stats(lib):
    """Bookkeeping of the factorisation schedule: with complex128 factors a
    level's first panel is always factored by a launch of its own, so at
    most panel_blocks - nfronts blocks are fused (lookahead); complex64
    factors also run the upper levels as panel-strip launches, which factor
    first panels too; the fused launches carry part of the update flops;
    and smaller update tiles (more workgroups per launch) never fuse more,
    since fusion needs every workgroup of the launch resident."""
    p64 = L.Plan(256, 2).stats()
    assert 0 < p64["fused_blocks"] <= p64["panel_blocks"] - p64["nfronts"]
    p = L.Plan(256, 2, precision="mixed")
    s = p.stats()
    assert p64["fused_blocks"] < s["fused_blocks"] <= s["panel_blocks"]
    assert 0 < s["fused_update_flops"] < s["update_flops"]
    nl = s["nlevels"]
    fused = {}
    for t in (32, 64, 128):
        p.set_tiles([t] * nl)
        fused[t] = p.stats()["fused_blocks"]
    assert fused[32] <= fused[64] <= fused[128]
    # n = 8 in 2D is a single front of 64 pivots (two panels, no boundary):
    # the second panel's block is factored inside the first panel's update,
    # which is the only update with any flops: 8 x 32^2 x 32
    q = L.Plan(8, 2).stats()
    assert q["nfronts"] == 1 and q["max_pivots"] == 64 and q["panel_blocks"] == 2
    assert q["fused_blocks"] == 1
    assert q["fused_update_flops"] == q["update_flops"] == 8 * 32 ** 2 * 32
    # complex64: a one-front level is a strip level, so both blocks are
    # factored by the strip launches
    q = L.Plan(8, 2, precision="mixed").stats()
    assert q["fused_blocks"] == 2 and q["fused_update_flops"] == q["update_flops"]


def test_pair_update_stats(lib):
    """Levels of fronts with at least 512 rows (not panel-strip levels) run
    the two-panel schedule: its products (pair_update, cross_update) are a
    part of update_flops disjoint from the lookahead launches'; the cross
    products (rank 32 over two 32-wide strips) are far smaller than the
    pair products on large fronts; plans without such fronts have none."""
    for n, d, prec in ((1024, 2, "mixed"), (1024, 2, "fp64"), (32, 3, "fp64"), (64, 3, "mixed")):
        s = L.Plan(n, d, precision=prec).stats()
        assert s["pair_update_flops"] > 0 and s["cross_update_flops"] > 0, (n, d, prec)
        assert s["cross_update_flops"] < 0.2 * s["pair_update_flops"], (n, d, prec)
        assert (s["pair_update_flops"] + s["cross_update_flops"] + s["fused_update_flops"]
                <= s["update_flops"] * (1 + 1e-12)), (n, d, prec)
    s = L.Plan(64, 2).stats()  # largest front 96 rows
    assert s["max_front"] < 512 and s["pair_update_flops"] == s["cross_update_flops"] == 0


def test_tile_cache_round_trip(lib, tmp_path):
    """A tile table written with lsp_plan_save_tiles is picked up by plans of
    the same (n, d, precision) created with tile_cache; other keys keep their
    default, saving again replaces the line, and malformed lines and a
    missing file are ignored."""
    path = str(tmp_path / "tiles.txt")
    p = L.Plan(64, 2, precision="mixed")
    default = p.tiles()
    tuned = [32 if i % 2 else 128 for i in range(len(default))]
    p.set_tiles(tuned)
    p.save_tiles(path)
    assert L.Plan(64, 2, precision="mixed", tile_cache=path).tiles() == tuned
    assert L.Plan(64, 2, precision="fp64", tile_cache=path).tiles() == L.Plan(64, 2, precision="fp64").tiles()
    assert L.Plan(32, 2, precision="mixed", tile_cache=path).tiles() == L.Plan(32, 2, precision="mixed").tiles()
    q = L.Plan(32, 2, precision="mixed")
    q.set_tiles([64] * len(q.tiles()))
    q.save_tiles(path)
    p.set_tiles(default)
    p.save_tiles(path)          # replaces the (64, 2, mixed) line
    lines = open(path).read().splitlines()
    assert len(lines) == 2
    assert L.Plan(64, 2, precision="mixed", tile_cache=path).tiles() == default
    assert L.Plan(32, 2, precision="mixed", tile_cache=path).tiles() == [64] * len(q.tiles())
    with open(path, "a") as f:
        f.write("64 2 1 not numbers\n")
    assert L.Plan(64, 2, precision="mixed", tile_cache=path).tiles() == default
    assert L.Plan(64, 2, precision="mixed", tile_cache=str(tmp_path / "absent.txt")).tiles() == default


def test_default_tiles_by_precision(lib):
    """Default trailing-update tiles: complex128 factors 32 on every level;
    complex64 ones 64, except in 2D up to 160 rows and above 512 rows (32)
    and a single 2D root front of 1024 rows or more (128)."""
    p64 = L.Plan(1024, 2, precision="fp64")
    assert set(p64.tiles()) == {32}
    pm = L.Plan(1024, 2, precision="mixed")
    t = pm.tiles()
    assert t[0] == 32 and t[-1] == 128 and set(t) == {32, 64, 128}
    assert L.Plan(256, 2, precision="mixed").tiles()[-1] == 64  # root of 257 rows
    t3 = L.Plan(64, 3, precision="mixed").tiles()
    assert set(t3) == {64}


def test_self_term_option_validated(lib):
    with pytest.raises(L.LspError):
        L.Plan(32, 2, self_term=3)
    L.Plan(32, 2, self_term=1)
    L.Plan(32, 2, self_term=2)
    with pytest.raises(L.LspError):
        L.self_term(1 / 32, 0.0, 2, 2)  # no 2D Laplace kernel


@pytest.mark.parametrize("n,d,omega", [(32, 2, 8 * np.pi), (256, 2, 64 * np.pi), (16, 3, 4 * np.pi),
                                       (96, 3, 24 * np.pi), (48, 3, 0.0)])
def test_host_self_terms_match_oracle(lib, n, d, omega):
    """The library's host self terms (Section 2.1's k_0) against the
    oracle's: the disk / ball closed forms and the cell integral to 1e-13,
    the fitted one-point correction (own e^{-x} Ei(x), Dawson, symmetric
    lattice sum, against mpmath / scipy and the full lattice) to 2e-12."""
    from oracle.greens import self_term
    h = 1.0 / n
    for mode, tol in ((0, 1e-13), (1, 1e-13), (2, 2e-12)):
        if mode == 1 and omega == 0:
            continue
        a, b = L.self_term(h, omega, d, mode), self_term(h, omega, d, mode)
        assert abs(a - b) <= tol * abs(b), (mode, a, b)


def test_laplace_options_validated(lib):
    """The Laplace equation (Section 5) is three-dimensional, and its set-up
    takes omega = 0 (the Helmholtz one omega > 0); both checked before any
    HIP call."""
    import ctypes
    with pytest.raises(L.LspError) as e:
        L.Plan(16, 2, equation="laplace")
    assert "three-dimensional" in str(e.value)
    p = L.Plan(8, 3, equation="laplace")
    h = ctypes.c_void_p()
    st = lib.lsp_setup(p._h, 1.0, ctypes.c_void_p(8), ctypes.c_void_p(8), 1 << 40, None, ctypes.byref(h))
    assert st == 1
    buf = ctypes.create_string_buffer(256)
    lib.lsp_last_error(buf, 256)
    assert b"omega must be 0" in buf.value
    q = L.Plan(8, 3)
    assert lib.lsp_setup(q._h, 0.0, ctypes.c_void_p(8), ctypes.c_void_p(8), 1 << 40, None, ctypes.byref(h)) == 1


def test_general_plan_classification(lib):
    """A general-domain plan (Section 4) classifies the points of Omega like
    the oracle: the same domain and boundary points; a rectangle plan
    reports the whole grid; invalid masks and options are refused."""
    import synth
    from oracle.general import classify
    for key in ("g1", "g1d", "g3"):
        w = synth.workload(key)
        n, d = w["n"], w["d"]
        s = L.Plan(n, d, mask=w["mask"]).stats()
        pts, _, interior = classify(w["mask"], n, d)
        assert s["domain_points"] == pts.size
        assert s["boundary_points"] == int(np.sum(~interior))
        assert s["sketch_cols"] == 2 * 3 ** d == w["R"].shape[0]
    s = L.Plan(16, 2).stats()
    assert s["domain_points"] == 256 and s["boundary_points"] == 0 and s["sketch_cols"] == 0
    assert L.Plan(16, 2, mask=np.ones(256, bool), sketch_cols=5).stats()["sketch_cols"] == 5
    with pytest.raises(L.LspError):
        L.Plan(16, 2, mask=np.zeros(256, bool))
    with pytest.raises(L.LspError):
        L.Plan(16, 3, mask=np.ones(16 ** 3, bool), equation="laplace")
    with pytest.raises(L.LspError):
        L.Plan(16, 2, mask=np.ones(256, bool), sketch_cols=5000)
    with pytest.raises(ValueError):
        L.Plan(16, 2, mask=np.ones(100, bool))
