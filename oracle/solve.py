"""End-to-end oracle pipeline: setup, factor, preconditioned GMRES solve."""
import numpy as np

from .greens import kernel_table
from .operator import Operator
from .stencil import all_stencils
from .sparse import build_QM, Preconditioner
from .gmres import gmres


class OracleProblem:
    """Helmholtz (omega > 0, medium m) or, with omega = 0 and potential V,
    Section 5's Laplace case (eq:lslap)."""

    def __init__(self, n, d, omega, m, b=2, self_term=0, potential=None):
        self.n, self.d, self.omega, self.b = n, d, float(omega), b
        self.m = np.asarray(m, dtype=np.float64) if m is not None else None
        self.ktab = kernel_table(n, d, omega, self_term)
        self.op = Operator(n, d, omega, self.m, self.ktab, potential=potential)
        self.stencils = all_stencils(self.ktab, d, n, b)
        self.Q, self.M = build_QM(n, d, omega, self.m, self.stencils, potential=potential)
        self.P = Preconditioner(self.Q, self.M)

    def rhs(self, uI):
        return self.op.rhs(uI)

    def solve_source(self, f, tol=1e-8, restart=30, max_iters=1000):
        """u + K(V u) = K f (eq:lslap)."""
        return self.solve_g(self.op.rhs_source(f), tol, restart, max_iters)

    def solve_g(self, g, tol=1e-8, restart=30, max_iters=1000):
        return gmres(self.op.apply, self.P, g, tol, restart, max_iters)

    def solve(self, uI, tol=1e-8, restart=30, max_iters=1000):
        return self.solve_g(self.rhs(uI), tol, restart, max_iters)
