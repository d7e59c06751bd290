"""Sparse stencil matrices Q and M and the preconditioner (oracle).

Section 2.2, eq:PCapp / eq:PC and Section 3.1 eq:ABop:
  Q = [A; B]      row i: Q(i, i+s) = alpha_{c(i)}(s) for s in mu_{c(i)}
  M = [A + C w^2 m; B]  (Section 5's Laplace case: V in place of w^2 m)
     interior row i: M(i, i+s) = alpha(s) + C(s) w^2 m_{i+s}
     boundary row i: M(i, :) = B(i, :) = Q(i, :)
  preconditioner: v -> M^{-1} (Q v).
Reading: m is used as given (not forced to zero near the boundary); that
only changes the quality of the boundary rows, not the solution of the
discrete system.  M^{-1} comes from scipy's SuperLU (COLAMD ordering,
threshold partial pivoting); M^{-1} is unique, so any ordering or pivoting
yields the same operator.
"""
import numpy as np
import scipy.sparse as sps
import scipy.sparse.linalg as spla

from .stencil import point_class, interior_class


def _neighbour(n, d, offsets):
    """For each grid point and each offset: neighbour linear index or -1."""
    N = n ** d
    idx = np.arange(N)
    I = np.stack([(idx // n ** a) % n for a in range(d)], axis=1)
    out = np.empty((N, offsets.shape[0]), dtype=np.int64)
    for k, s in enumerate(offsets):
        J = I + s
        ok = np.all((J >= 0) & (J < n), axis=1)
        lin = np.sum(J * (n ** np.arange(d)), axis=1)
        out[:, k] = np.where(ok, lin, -1)
    return out


def build_QM(n, d, omega, m, stencils, potential=None):
    N = n ** d
    cls = point_class(n, d)
    ic = interior_class(d)
    rows_q, cols_q, vals_q = [], [], []
    rows_m, cols_m, vals_m = [], [], []
    w2m = (np.asarray(potential, dtype=np.float64) if potential is not None
           else omega ** 2 * np.asarray(m, dtype=np.float64))
    for st in stencils:
        pts = np.nonzero(cls == st.c)[0]
        if pts.size == 0:
            continue
        nb = _neighbour(n, d, st.offsets)[pts]
        assert np.all(nb >= 0), "class stencil leaves the domain"
        for k in range(st.offsets.shape[0]):
            j = nb[:, k]
            rows_q.append(pts); cols_q.append(j)
            vals_q.append(np.full(pts.size, st.alpha[k]))
            rows_m.append(pts); cols_m.append(j)
            if st.c == ic:
                vals_m.append(st.alpha[k] + st.C[k] * w2m[j])
            else:
                vals_m.append(np.full(pts.size, st.alpha[k]))
    Q = sps.csr_matrix((np.concatenate(vals_q), (np.concatenate(rows_q), np.concatenate(cols_q))),
                       shape=(N, N), dtype=np.complex128)
    M = sps.csr_matrix((np.concatenate(vals_m), (np.concatenate(rows_m), np.concatenate(cols_m))),
                       shape=(N, N), dtype=np.complex128)
    return Q, M


class Preconditioner:
    """v -> M^{-1} Q v with a sparse LU of M."""

    def __init__(self, Q, M):
        self.Q = Q
        self.M = M
        self.lu = spla.splu(M.tocsc())

    def solve_M(self, z):
        return self.lu.solve(np.asarray(z, dtype=np.complex128))

    def __call__(self, v):
        return self.lu.solve(self.Q @ np.asarray(v, dtype=np.complex128))
