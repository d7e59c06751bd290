"""General domains (Section 4): the sparsifying preconditioner when the
support Omega of m is not a rectangle (oracle; test infrastructure).

The unknowns are the grid points of Omega (a mask over the n^d box of the
rectangle case, same grid and kernel table).  The operator is the
restriction of eq:lso to Omega, A = I + K(Omega, Omega) w^2 m(Omega), and
the right-hand side g = K(-w^2 m u_I) restricted to Omega.

Rows of the sparse operators, per point i of Omega with neighbourhood
mu(i) = the 3^d block around i intersected with Omega:
  * interior points (the whole 3^d block lies in Omega): exactly the
    rectangle's interior rows (Section 3.1): Q(i, i+s) = alpha(s),
    M(i, i+s) = alpha(s) + C(s) w^2 m_{i+s}, with the interior class stencil
    of the n^d box;
  * boundary points (some neighbour outside Omega or outside the box): the
    row B(i, mu(i)) should nearly annihilate (K w^2 m)(mu(i), :).  Section 4
    sketches that matrix with an N x r Gaussian matrix R, T = (K w^2 m) R,
    and takes the unit row vector alpha minimising ||alpha T(mu(i), :)||:
    with T(mu(i), :) = U S V^* it is alpha = U(:, end)^*.  Then
    Q(i, mu(i)) = M(i, mu(i)) = alpha.
Readings: (i) R's rows outside Omega are not used (the columns of K w^2 m
are those of Omega); R is an input (seeded by the caller); r defaults to
2 * 3^d (the paper asks for a constant multiple of the stencil size).
(ii) mu(i) is listed in slot order q = sum_a (s_a + 1) 3^a, and alpha is
normalised like the rectangle's stencils: unit norm, centre entry real
positive.  (iii) A boundary row uses no C term, as the rectangle's B rows.
"""
import numpy as np
import scipy.sparse as sps

from .greens import kernel_table
from .operator import Operator
from .stencil import class_stencil, interior_class, slot
from .sparse import Preconditioner
from .gmres import gmres


def neighbour_offsets(d):
    """All 3^d offsets in slot order (axis 1 fastest), shape [3^d, d]."""
    q = np.arange(3 ** d)
    return np.stack([(q // 3 ** a) % 3 - 1 for a in range(d)], axis=1)


def classify(mask, n, d):
    """Points of Omega, and for each: its neighbours' linear indices per slot
    (-1 outside the box or outside Omega) and whether it is interior."""
    mask = np.asarray(mask, dtype=bool).reshape(-1)
    pts = np.nonzero(mask)[0]
    I = np.stack([(pts // n ** a) % n for a in range(d)], axis=1)
    offs = neighbour_offsets(d)
    nb = np.empty((pts.size, offs.shape[0]), dtype=np.int64)
    for k, s in enumerate(offs):
        J = I + s
        inbox = np.all((J >= 0) & (J < n), axis=1)
        lin = np.sum(np.where(inbox[:, None], J, 0) * (n ** np.arange(d)), axis=1)
        nb[:, k] = np.where(inbox & mask[lin], lin, -1)
    interior = np.all(nb >= 0, axis=1)
    return pts, nb, interior


def sketch(op, mask, R):
    """T = (K w^2 m) R over the columns of Omega: one K product per column of
    R (R given as [r, N] over the box; its rows outside Omega are zeroed)."""
    mask = np.asarray(mask, dtype=bool).reshape(-1)
    Rm = np.where(mask[None, :], np.asarray(R, dtype=np.float64), 0.0)
    return op.K(op.p[None, :] * Rm)  # [r, N]


def boundary_stencil(Tmu):
    """Unit alpha minimising ||alpha Tmu|| (Tmu: |mu| x r), and all singular
    values of Tmu (descending)."""
    U, sig, _ = np.linalg.svd(Tmu, full_matrices=False)
    return np.conj(U[:, -1]), sig


class GeneralStencils:
    """Per boundary point: its linear index, the slots of mu(i), alpha on
    those slots (slot-padded to 3^d, zero elsewhere) and the singular values."""

    def __init__(self, n, d, pts, nb, interior, T):
        self.centre = (3 ** d) // 2
        bpos = np.nonzero(~interior)[0]
        self.points = pts[bpos]
        self.alpha = np.zeros((bpos.size, 3 ** d), dtype=np.complex128)
        self.sigma = []
        self.slots = []
        for k, pos in enumerate(bpos):
            sl = np.nonzero(nb[pos] >= 0)[0]
            alpha, sig = boundary_stencil(T[:, nb[pos, sl]].T)
            c = int(np.nonzero(sl == self.centre)[0][0])
            alpha = alpha / (alpha[c] / abs(alpha[c]))
            self.alpha[k, sl] = alpha
            self.sigma.append(sig)
            self.slots.append(sl)

    @property
    def sigma_min(self):
        return np.array([s[-1] for s in self.sigma])


def build_QM_general(n, d, mask, p, interior_st, gst):
    """Q and M over the points of Omega (rows and columns in increasing
    linear index), p = w^2 m (or V)."""
    pts, nb, interior = classify(mask, n, d)
    pos = -np.ones(n ** d, dtype=np.int64)
    pos[pts] = np.arange(pts.size)
    offs = neighbour_offsets(d)
    isl = slot(interior_st.offsets)  # interior class offsets in slot order
    assert np.array_equal(isl, np.arange(3 ** d))
    rq, cq, vq, vm = [], [], [], []
    ip = np.nonzero(interior)[0]
    for k in range(offs.shape[0]):
        j = nb[ip, k]
        rq.append(ip); cq.append(pos[j])
        vq.append(np.full(ip.size, interior_st.alpha[k]))
        vm.append(interior_st.alpha[k] + interior_st.C[k] * p[j])
    bpos = pos[gst.points]
    for k in range(offs.shape[0]):
        has = nb[bpos, k] >= 0
        rq.append(bpos[has]); cq.append(pos[nb[bpos[has], k]])
        vq.append(gst.alpha[has, k]); vm.append(gst.alpha[has, k])
    shape = (pts.size, pts.size)
    rows, cols = np.concatenate(rq), np.concatenate(cq)
    Q = sps.csr_matrix((np.concatenate(vq), (rows, cols)), shape=shape, dtype=np.complex128)
    M = sps.csr_matrix((np.concatenate(vm), (rows, cols)), shape=shape, dtype=np.complex128)
    return Q, M


class GeneralProblem:
    """Section 4's preconditioned solve on the support Omega (a mask over
    the n^d grid) with the sketch R ([r, N] Gaussian, an input)."""

    def __init__(self, n, d, omega, m, mask, R, b=2, self_term=0):
        self.n, self.d, self.omega = n, d, float(omega)
        self.mask = np.asarray(mask, dtype=bool).reshape(-1)
        self.m = np.asarray(m, dtype=np.float64)
        self.ktab = kernel_table(n, d, omega, self_term)
        self.op = Operator(n, d, omega, self.m, self.ktab)
        self.pts, self.nb, self.interior = classify(self.mask, n, d)
        self.interior_st = class_stencil(self.ktab, interior_class(d), d, n, b)
        self.T = sketch(self.op, self.mask, R)
        self.gst = GeneralStencils(n, d, self.pts, self.nb, self.interior, self.T)
        self.Q, self.M = build_QM_general(n, d, self.mask, self.op.p, self.interior_st, self.gst)
        self.P = Preconditioner(self.Q, self.M)

    def to_box(self, x):
        """A vector over Omega as a box field (zero outside Omega)."""
        out = np.zeros(self.n ** self.d, dtype=np.complex128)
        out[self.pts] = x
        return out

    def apply(self, x):
        """(I + K w^2 m) restricted to Omega."""
        return x + self.op.K(self.op.p * self.to_box(x))[self.pts]

    def rhs(self, uI):
        return self.op.rhs(uI)[self.pts]

    def solve(self, uI, tol=1e-8, restart=30, max_iters=1000):
        """GMRES on Omega; result.x is over the points of Omega."""
        return gmres(self.apply, self.P, self.rhs(uI), tol, restart, max_iters)
