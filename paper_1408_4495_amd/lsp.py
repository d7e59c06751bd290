"""Thin ctypes binding of liblsp.so (the C ABI declared in include/lsp.h).

Argument marshalling only: torch tensors provide device memory (problem and
solve workspaces) and the HIP stream; every step of the solver runs in the
library's HIP kernels.  Importing this module does not need a GPU; creating a
Problem does, and fails loudly when the library has not been built.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblsp.so")

LSP_FP64, LSP_MIXED = 0, 1
LSP_RHS_INCIDENT, LSP_RHS_G, LSP_RHS_SOURCE = 0, 1, 2
LSP_HELMHOLTZ, LSP_LAPLACE = 0, 1
RHS_KINDS = {"incident": LSP_RHS_INCIDENT, "g": LSP_RHS_G, "source": LSP_RHS_SOURCE}
STATUS = {0: "LSP_OK", 1: "LSP_ERR_ARG", 2: "LSP_ERR_OOM", 3: "LSP_ERR_HIP",
          4: "LSP_ERR_STATE", 5: "LSP_ERR_SINGULAR", 6: "LSP_ERR_NOCONV"}
EXPORTED = ["lsp_options_default", "lsp_plan_create", "lsp_plan_destroy", "lsp_plan_stats_get",
            "lsp_plan_bytes", "lsp_setup", "lsp_problem_destroy", "lsp_factor", "lsp_solve",
            "lsp_apply_op", "lsp_apply_K", "lsp_apply_Q", "lsp_solve_M", "lsp_apply_precond",
            "lsp_get_kernel_table", "lsp_get_stencils", "lsp_get_matrix", "lsp_status_string",
            "lsp_last_error", "lsp_timing_enable", "lsp_timing_reset", "lsp_timing_count",
            "lsp_timing_get", "lsp_plan_get_tiles", "lsp_plan_set_tiles", "lsp_apply_op_noalloc", "lsp_plan_save_tiles",
            "lsp_plan_create_general", "lsp_setup_general", "lsp_get_boundary_stencils",
            "lsp_field_bytes", "lsp_exterior_field", "lsp_far_field", "lsp_self_term"]


class Options(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("restart", ctypes.c_int), ("max_iters", ctypes.c_int),
                ("precision", ctypes.c_int), ("buffer_b", ctypes.c_int), ("leaf", ctypes.c_int),
                ("panel", ctypes.c_int), ("dense_sweeps", ctypes.c_int), ("blocked_sweeps", ctypes.c_int),
                ("self_term", ctypes.c_int), ("equation", ctypes.c_int), ("tile_cache", ctypes.c_char_p)]


class RhsInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("converged", ctypes.c_int),
                ("relres_true", ctypes.c_double), ("relres_est", ctypes.c_double),
                ("t_setup", ctypes.c_double), ("t_factor", ctypes.c_double), ("t_solve", ctypes.c_double)]


class PlanStats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("d", ctypes.c_int), ("N", ctypes.c_int), ("L", ctypes.c_int),
                ("nfronts", ctypes.c_int), ("nlevels", ctypes.c_int), ("max_front", ctypes.c_int),
                ("max_pivots", ctypes.c_int), ("factor_entries", ctypes.c_double),
                ("front_entries", ctypes.c_double), ("factor_flops", ctypes.c_double),
                ("sweep_entries", ctypes.c_double), ("update_flops", ctypes.c_double),
                ("panel_blocks", ctypes.c_double),
                ("fused_blocks", ctypes.c_double), ("fused_update_flops", ctypes.c_double),
                ("dense_entries", ctypes.c_double), ("dense_levels", ctypes.c_int),
                ("blocked_levels", ctypes.c_int), ("blocked_entries", ctypes.c_double),
                ("chain_entries", ctypes.c_double), ("blocked_panel_entries", ctypes.c_double),
                ("trsm_flops", ctypes.c_double), ("assemble_entries", ctypes.c_double),
                ("mchain_levels", ctypes.c_int), ("mchain_entries", ctypes.c_double),
                ("pair_update_flops", ctypes.c_double), ("cross_update_flops", ctypes.c_double),
                ("mchain_pivots", ctypes.c_double), ("mchain_rows", ctypes.c_double),
                ("mchain_child_rows", ctypes.c_double),
                ("domain_points", ctypes.c_int), ("boundary_points", ctypes.c_int), ("sketch_cols", ctypes.c_int)]


class LspError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load():
    """Load liblsp.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1408_4495_amd.build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp, sz, ci, cd = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_double
    sigs = {
        "lsp_options_default": [ctypes.POINTER(Options)],
        "lsp_plan_create": [ci, ci, ci, ctypes.POINTER(Options), ctypes.POINTER(vp)],
        "lsp_plan_create_general": [ci, ci, ci, ctypes.POINTER(Options), vp, ci, ctypes.POINTER(vp)],
        "lsp_setup_general": [vp, cd, vp, vp, vp, sz, vp, ctypes.POINTER(vp)],
        "lsp_get_boundary_stencils": [vp, vp, vp, vp],
        "lsp_field_bytes": [vp, ci, ctypes.POINTER(sz)],
        "lsp_self_term": [cd, cd, ci, ci, ctypes.POINTER(cd)],
        "lsp_exterior_field": [vp, ci, vp, vp, ci, vp, vp, vp, sz],
        "lsp_far_field": [vp, ci, vp, vp, ci, vp, vp, vp, sz],
        "lsp_plan_stats_get": [vp, ctypes.POINTER(PlanStats)],
        "lsp_plan_bytes": [vp, ci, ci, ctypes.POINTER(sz), ctypes.POINTER(sz)],
        "lsp_setup": [vp, cd, vp, vp, sz, vp, ctypes.POINTER(vp)],
        "lsp_factor": [vp],
        "lsp_solve": [vp, ci, ci, vp, vp, vp, sz, ctypes.POINTER(RhsInfo)],
        "lsp_apply_op": [vp, ci, ci, vp, vp, vp, sz],
        "lsp_apply_K": [vp, ci, ci, vp, vp, vp, sz],
        "lsp_apply_op_noalloc": [vp, ci, ci, vp, vp],
        "lsp_apply_Q": [vp, ci, vp, vp],
        "lsp_solve_M": [vp, ci, vp, vp, vp, sz],
        "lsp_apply_precond": [vp, ci, vp, vp, vp, sz],
        "lsp_get_kernel_table": [vp, vp],
        "lsp_get_stencils": [vp, vp, vp, vp],
        "lsp_get_matrix": [vp, vp],
        "lsp_plan_get_tiles": [vp, ctypes.POINTER(ci), ci],
        "lsp_plan_set_tiles": [vp, ctypes.POINTER(ci), ci],
        "lsp_plan_save_tiles": [vp, ctypes.c_char_p],
    }
    for name, args in sigs.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ci
    lib.lsp_plan_destroy.argtypes = [vp]
    lib.lsp_plan_destroy.restype = None
    lib.lsp_problem_destroy.argtypes = [vp]
    lib.lsp_problem_destroy.restype = None
    lib.lsp_status_string.argtypes = [ci]
    lib.lsp_status_string.restype = ctypes.c_char_p
    lib.lsp_last_error.argtypes = [ctypes.c_char_p, sz]
    lib.lsp_last_error.restype = None
    lib.lsp_timing_enable.argtypes = [ci]
    lib.lsp_timing_enable.restype = ci
    lib.lsp_timing_reset.argtypes = []
    lib.lsp_timing_reset.restype = ci
    lib.lsp_timing_count.argtypes = []
    lib.lsp_timing_count.restype = ci
    lib.lsp_timing_get.argtypes = [ci, ctypes.c_char_p, sz, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_longlong)]
    lib.lsp_timing_get.restype = ci
    _lib = lib
    return lib


def _check(status):
    if status != 0:
        buf = ctypes.create_string_buffer(1024)
        _lib.lsp_last_error(buf, 1024)
        raise LspError(status, buf.value.decode(errors="replace"))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def self_term(h, omega, d, mode=0):
    """k_0 of the kernel table (see lsp.h, lsp_self_term), host computation."""
    out = (ctypes.c_double * 2)()
    _check(load().lsp_self_term(float(h), float(omega), int(d), int(mode), out))
    return complex(out[0], out[1])


def timing_enable(on=True):
    """Bracket every library kernel launch with HIP events (see lsp.h)."""
    _check(load().lsp_timing_enable(1 if on else 0))


def timing_reset():
    _check(load().lsp_timing_reset())


def timing_read():
    """{kernel name: (total ms, launches)} recorded since the last reset."""
    lib = load()
    n = lib.lsp_timing_count()
    if n < 0:
        raise LspError(3, "HIP error while reading kernel timings")
    out = {}
    buf = ctypes.create_string_buffer(256)
    for i in range(n):
        ms, cnt = ctypes.c_double(), ctypes.c_longlong()
        _check(lib.lsp_timing_get(i, buf, 256, ctypes.byref(ms), ctypes.byref(cnt)))
        out[buf.value.decode()] = (ms.value, cnt.value)
    return out


class Plan:
    """Symbolic plan for an n^d grid (host-side nested dissection).  With a
    mask (n^d booleans), a general-domain plan (Section 4) whose unknowns
    are the points of Omega; sketch_cols = r (0: 2 * 3^d)."""

    def __init__(self, n, d, max_nrhs=1, tol=1e-8, restart=30, max_iters=1000, precision="fp64",
                 buffer_b=2, leaf=0, panel=0, dense_sweeps=1, blocked_sweeps=1, self_term=0,
                 tile_cache=None, equation="helmholtz", mask=None, sketch_cols=0):
        lib = load()
        o = Options()
        _check(lib.lsp_options_default(ctypes.byref(o)))
        o.tol, o.restart, o.max_iters = tol, restart, max_iters
        o.precision = LSP_MIXED if precision in ("mixed", LSP_MIXED) else LSP_FP64
        o.buffer_b, o.leaf, o.panel, o.dense_sweeps = buffer_b, leaf, panel, dense_sweeps
        o.blocked_sweeps = blocked_sweeps
        o.self_term = self_term
        o.equation = LSP_LAPLACE if equation in ("laplace", LSP_LAPLACE) else LSP_HELMHOLTZ
        o.tile_cache = None if tile_cache is None else os.fsencode(tile_cache)
        self.opts = o
        self.n, self.d, self.max_nrhs = n, d, max_nrhs
        self.precision = o.precision
        h = ctypes.c_void_p()
        self.general = mask is not None
        if self.general:
            mk = np.ascontiguousarray(np.asarray(mask).reshape(-1) != 0, dtype=np.uint8)
            if mk.size != n ** d:
                raise ValueError("mask has the wrong length")
            _check(lib.lsp_plan_create_general(n, d, max_nrhs, ctypes.byref(o), mk.ctypes.data_as(ctypes.c_void_p),
                                               int(sketch_cols), ctypes.byref(h)))
        else:
            _check(lib.lsp_plan_create(n, d, max_nrhs, ctypes.byref(o), ctypes.byref(h)))
        self._h = h

    def bytes(self, nrhs=1, precision=None):
        prec = self.precision if precision is None else precision
        pb, sb = ctypes.c_size_t(), ctypes.c_size_t()
        _check(_lib.lsp_plan_bytes(self._h, prec, nrhs, ctypes.byref(pb), ctypes.byref(sb)))
        return pb.value, sb.value

    def tiles(self):
        nl = self.stats()["nlevels"]
        arr = (ctypes.c_int * nl)()
        _check(_lib.lsp_plan_get_tiles(self._h, arr, nl))
        return list(arr)

    def set_tiles(self, tiles):
        arr = (ctypes.c_int * len(tiles))(*tiles)
        _check(_lib.lsp_plan_set_tiles(self._h, arr, len(tiles)))

    def save_tiles(self, path):
        """Write this plan's tile table to the cache file `path`."""
        _check(_lib.lsp_plan_save_tiles(self._h, os.fsencode(path)))

    def stats(self):
        s = PlanStats()
        _check(_lib.lsp_plan_stats_get(self._h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in PlanStats._fields_}

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.lsp_plan_destroy(self._h)
            self._h = None


class Problem:
    """Set-up (kernel table, spectrum, stencils, M) on the GPU; factor; solve.

    m: real medium of length n^d (numpy or torch), or for a Laplace plan the
    potential V (with omega = 0); R: the [r, n^d] real sketch of a
    general-domain plan (Section 4); device memory comes from torch; work is
    enqueued on `stream` (default: torch's current stream)."""

    def __init__(self, plan, omega, m, device="cuda:0", stream=None, R=None):
        import torch
        self.torch = torch
        self.plan = plan
        self.device = torch.device(device)
        if not torch.cuda.is_available():
            raise RuntimeError("a GPU is required")
        lib = load()
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        N = plan.n ** plan.d
        # every allocation below is made on the problem's stream, so torch's
        # caching allocator reuses its memory only after that stream's work
        with torch.cuda.device(self.device), torch.cuda.stream(self.stream):
            m_t = torch.as_tensor(np.asarray(m, dtype=np.float64) if not isinstance(m, torch.Tensor) else m)
            m_t = m_t.to(device=self.device, dtype=torch.float64).contiguous()
            if m_t.numel() != N:
                raise ValueError("medium has the wrong length")
            pbytes, _ = plan.bytes(1)
            self.ws = torch.empty(pbytes, dtype=torch.uint8, device=self.device)
            self._solve_ws = None
            h = ctypes.c_void_p()
            if getattr(plan, "general", False):
                if R is None:
                    raise ValueError("a general-domain plan needs the sketch R")
                r = plan.stats()["sketch_cols"]
                R_t = torch.as_tensor(np.asarray(R, dtype=np.float64) if not isinstance(R, torch.Tensor) else R)
                R_t = R_t.to(device=self.device, dtype=torch.float64).contiguous()
                if R_t.numel() != r * N:
                    raise ValueError(f"sketch must be [{r}, {N}]")
                _check(lib.lsp_setup_general(plan._h, float(omega), _ptr(m_t), _ptr(R_t), _ptr(self.ws), pbytes,
                                             ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
            else:
                _check(lib.lsp_setup(plan._h, float(omega), _ptr(m_t), _ptr(self.ws), pbytes,
                                     ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self.omega = float(omega)
        self.N = N
        self._phases = {}

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.lsp_problem_destroy(self._h)
            self._h = None

    # -- helpers
    def _ctx(self):
        """Device and stream context of the problem: tensors created inside
        belong to the problem's stream."""
        import contextlib
        stack = contextlib.ExitStack()
        stack.enter_context(self.torch.cuda.device(self.device))
        stack.enter_context(self.torch.cuda.stream(self.stream))
        return stack

    def _handoff(self, *ts):
        """Make the caller's current stream wait for the problem's stream
        before it uses the returned tensors."""
        cur = self.torch.cuda.current_stream(self.device)
        if cur != self.stream:
            ev = self.torch.cuda.Event()
            ev.record(self.stream)
            cur.wait_event(ev)
        return ts[0] if len(ts) == 1 else ts

    def _work(self, nrhs):
        _, sb = self.plan.bytes(nrhs)
        if self._solve_ws is None or self._solve_ws.numel() < sb:
            self._solve_ws = self.torch.empty(sb, dtype=self.torch.uint8, device=self.device)
        return self._solve_ws

    def _field(self, x):
        t = self.torch
        x = t.as_tensor(x) if not isinstance(x, t.Tensor) else x
        x = x.to(device=self.device, dtype=t.complex128).contiguous()
        if x.dim() == 1:
            x = x.reshape(1, -1)
        if x.shape[1] != self.N:
            raise ValueError("field has the wrong length")
        return x

    # -- API
    def factor(self):
        _check(_lib.lsp_factor(self._h))

    def solve(self, rhs, kind="incident"):
        with self._ctx():
            x = self._field(rhs)
            nrhs = x.shape[0]
            u = self.torch.empty_like(x)
            ws = self._work(nrhs)
            info = (RhsInfo * nrhs)()
            k = RHS_KINDS[kind]
            st = _lib.lsp_solve(self._h, nrhs, k, _ptr(x), _ptr(u), _ptr(ws), ws.numel(), info)
        infos = [{"iters": i.iters, "converged": bool(i.converged), "relres_true": i.relres_true,
                  "relres_est": i.relres_est, "t_setup": i.t_setup, "t_factor": i.t_factor,
                  "t_solve": i.t_solve} for i in info]
        if infos:
            self._phases = {"setup": infos[0]["t_setup"], "factor": infos[0]["t_factor"],
                            "solve": infos[0]["t_solve"]}
        if st != 0 and st != 6:
            _check(st)
        return u, infos, st

    def phase_ms(self):
        """Device milliseconds of set-up, the last factorisation and the last
        solve (the library's HIP events on the problem's stream)."""
        return dict(self._phases)

    def apply_op(self, x, precision=LSP_FP64):
        with self._ctx():
            x = self._field(x)
            y = self.torch.empty_like(x)
            ws = self._work(x.shape[0])
            _check(_lib.lsp_apply_op(self._h, x.shape[0], precision, _ptr(x), _ptr(y), _ptr(ws), ws.numel()))
        return self._handoff(y)

    def apply_op_noalloc(self, x, precision=LSP_FP64):
        """y = x + K(w^2 m x) with the library's static scratch (no workspace)."""
        with self._ctx():
            x = self._field(x)
            y = self.torch.empty_like(x)
            _check(_lib.lsp_apply_op_noalloc(self._h, x.shape[0], precision, _ptr(x), _ptr(y)))
        return self._handoff(y)

    def apply_K(self, x, precision=LSP_FP64):
        with self._ctx():
            x = self._field(x)
            y = self.torch.empty_like(x)
            ws = self._work(x.shape[0])
            _check(_lib.lsp_apply_K(self._h, x.shape[0], precision, _ptr(x), _ptr(y), _ptr(ws), ws.numel()))
        return self._handoff(y)

    def apply_Q(self, x):
        with self._ctx():
            x = self._field(x)
            y = self.torch.empty_like(x)
            _check(_lib.lsp_apply_Q(self._h, x.shape[0], _ptr(x), _ptr(y)))
        return self._handoff(y)

    def solve_M(self, z):
        with self._ctx():
            z = self._field(z)
            x = self.torch.empty_like(z)
            ws = self._work(z.shape[0])
            _check(_lib.lsp_solve_M(self._h, z.shape[0], _ptr(z), _ptr(x), _ptr(ws), ws.numel()))
        return self._handoff(x)

    def apply_precond(self, v):
        with self._ctx():
            v = self._field(v)
            x = self.torch.empty_like(v)
            ws = self._work(v.shape[0])
            _check(_lib.lsp_apply_precond(self._h, v.shape[0], _ptr(v), _ptr(x), _ptr(ws), ws.numel()))
        return self._handoff(x)

    def kernel_table(self):
        t = self.torch
        with self._ctx():
            k = t.empty((self.plan.n + 1) ** self.plan.d, dtype=t.complex128, device=self.device)
            _check(_lib.lsp_get_kernel_table(self._h, _ptr(k)))
        return self._handoff(k)

    def stencils(self):
        nc = 3 ** self.plan.d
        alpha = np.zeros(nc * 27, dtype=np.complex128)
        C = np.zeros(nc * 27, dtype=np.complex128)
        sigma = np.zeros(nc * 27, dtype=np.float64)
        _check(_lib.lsp_get_stencils(self._h, alpha.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     sigma.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     C.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return alpha.reshape(nc, 27), sigma.reshape(nc, 27), C.reshape(nc, 27)

    def _eval_field(self, fn, u, uI, pts):
        t = self.torch
        with self._ctx():
            u = self._field(u)
            uI = self._field(uI)
            if u.shape != uI.shape:
                raise ValueError("u and u_I must have the same shape")
            P = t.as_tensor(np.asarray(pts, dtype=np.float64) if not isinstance(pts, t.Tensor) else pts)
            P = P.to(device=self.device, dtype=t.float64).reshape(-1, self.plan.d).contiguous()
            npts = P.shape[0]
            nb = ctypes.c_size_t()
            _check(_lib.lsp_field_bytes(self.plan._h, npts, ctypes.byref(nb)))
            ws = t.empty(nb.value, dtype=t.uint8, device=self.device)
            out = t.empty((u.shape[0], npts), dtype=t.complex128, device=self.device)
            _check(fn(self._h, u.shape[0], _ptr(u), _ptr(uI), npts, _ptr(P), _ptr(out), _ptr(ws), nb.value))
        return self._handoff(out)

    def exterior_field(self, u, uI, points):
        """Scattered field at points [P, d] (Section 1's representation; see
        lsp.h): [nrhs, P] complex128."""
        return self._eval_field(_lib.lsp_exterior_field, u, uI, points)

    def far_field(self, u, uI, dirs):
        """Far-field pattern at unit directions [P, d]: [nrhs, P]."""
        return self._eval_field(_lib.lsp_far_field, u, uI, dirs)

    def boundary_stencils(self):
        """General domains: (points [nbnd] int, alpha [nbnd, 27] complex,
        sigma [nbnd, 27]) of the boundary points (see lsp.h)."""
        nb = self.plan.stats()["boundary_points"]
        pts = np.zeros(max(nb, 1), dtype=np.int32)
        alpha = np.zeros(max(nb, 1) * 27, dtype=np.complex128)
        sigma = np.zeros(max(nb, 1) * 27, dtype=np.float64)
        _check(_lib.lsp_get_boundary_stencils(self._h, pts.ctypes.data_as(ctypes.c_void_p),
                                              alpha.ctypes.data_as(ctypes.c_void_p),
                                              sigma.ctypes.data_as(ctypes.c_void_p)))
        return pts[:nb], alpha.reshape(-1, 27)[:nb], sigma.reshape(-1, 27)[:nb]

    def matrix(self):
        t = self.torch
        ns = 3 ** self.plan.d
        with self._ctx():
            M = t.empty((self.N, ns), dtype=t.complex128, device=self.device)
            _check(_lib.lsp_get_matrix(self._h, _ptr(M)))
        return self._handoff(M)
