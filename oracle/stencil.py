"""Stencil classes and their null vectors (oracle; test infrastructure).

Section 2.2: the neighbourhood mu(i) is the infinity-ball of radius 1 around
grid point i, clipped to the domain; a point is interior when mu(i) is the
full 3^d block.  Section 3.1 (2D) and its 3D list: on the rectangle the rows
of A (interior) and B (boundary) are translation-invariant within each of the
3^d position classes, and each class's stencil alpha is the unit vector that
minimises ||alpha K(mu_c(0), F_c)|| over a far set F_c (eq:Fmin, eq:Emin,
eq:Cmin): alpha = U(:, end)^* from the SVD K(mu_c(0), F_c) = U S V^*.

Per axis a point is Lo (i_a = 0), Mid, or Hi (i_a = n-1).  Per axis the
translated stencil offsets are Lo {0,1}, Mid {-1,0,1}, Hi {-1,0}, and the far
set is the open integer interval Lo (b, n), Mid (-n, n), Hi (-n, -b); the
far set is their product, and for the all-Mid (interior) class mu(0) itself
is removed, as in I_n.  The paper derives one edge and one corner ("suppose
the right one"); reading: every class is computed the same way, so mirror
classes come out as mirror stencils.

Readings: (i) the singular vector is fixed up to a unit scalar; alpha is
normalised so ||alpha|| = 1 and its centre (offset 0) entry is real positive.
The preconditioner M^{-1} Q is unchanged by any per-row scalar.  (ii) b is
not given; it is a parameter, default 2.  The 3D corner set's "x_1 = 2" is
read as the corner x_1 = x_2 = x_3 = 1.

Class id: c = sum_a cls_a 3^a with cls 0 = Lo, 1 = Mid, 2 = Hi, axis 1 least
significant.  Offsets inside a class are listed with axis 1 fastest.  The
padded 3^d slot of an offset s is q = sum_a (s_a + 1) 3^a.
"""
import itertools
import numpy as np

LO, MID, HI = 0, 1, 2
AXIS_OFFSETS = {LO: (0, 1), MID: (-1, 0, 1), HI: (-1, 0)}


def class_tuple(c, d):
    return tuple((c // 3 ** a) % 3 for a in range(d))


def interior_class(d):
    return sum(MID * 3 ** a for a in range(d))


def class_offsets(c, d):
    """Stencil offsets of class c, shape [s_c, d], axis 1 fastest."""
    ct = class_tuple(c, d)
    per_axis = [AXIS_OFFSETS[ct[a]] for a in range(d)]
    # itertools.product varies the last factor fastest: feed axes reversed
    rows = [tuple(reversed(p)) for p in itertools.product(*reversed(per_axis))]
    return np.array(rows, dtype=np.int64)


def far_set(c, d, n, b):
    """Translated far set F_c, shape [|F_c|, d]."""
    ct = class_tuple(c, d)
    rng = []
    for a in range(d):
        if ct[a] == LO:
            rng.append(np.arange(b + 1, n))
        elif ct[a] == MID:
            rng.append(np.arange(-n + 1, n))
        else:
            rng.append(np.arange(-n + 1, -b))
    mesh = np.meshgrid(*rng, indexing="ij")
    F = np.stack([g.reshape(-1) for g in mesh], axis=1)
    if c == interior_class(d):
        F = F[np.max(np.abs(F), axis=1) > 1]
    return F


def slot(offsets):
    """Padded 3^d slot index of each offset row."""
    offsets = np.atleast_2d(offsets)
    return np.sum((offsets + 1) * (3 ** np.arange(offsets.shape[1])), axis=1)


def kernel_block(ktab, S, J):
    """K(S, J) with K(s, j) = k_{s-j} read from the |t| table."""
    T = np.abs(S[:, None, :] - J[None, :, :])
    return ktab[tuple(T[..., a] for a in range(S.shape[1]))]


class StencilClass:
    def __init__(self, c, offsets, alpha, sigma, C):
        self.c = c
        self.offsets = offsets       # [s, d]
        self.alpha = alpha           # [s] complex, unit norm, centre real > 0
        self.sigma = sigma           # all singular values, descending
        self.C = C                   # [s] complex: alpha K(mu_c, mu_c)

    @property
    def sigma_min(self):
        return self.sigma[-1]


def class_stencil(ktab, c, d, n, b):
    """Null vector of K(mu_c(0), F_c) by dense SVD, and C_c = alpha K(mu, mu)."""
    S = class_offsets(c, d)
    F = far_set(c, d, n, b)
    X = kernel_block(ktab, S, F)
    U, sig, _ = np.linalg.svd(X, full_matrices=False)
    alpha = np.conj(U[:, -1])
    centre = int(np.nonzero(np.all(S == 0, axis=1))[0][0])
    ph = alpha[centre] / abs(alpha[centre])
    alpha = alpha / ph
    C = alpha @ kernel_block(ktab, S, S)
    return StencilClass(c, S, alpha, sig, C)


def all_stencils(ktab, d, n, b=2):
    return [class_stencil(ktab, c, d, n, b) for c in range(3 ** d)]


def point_class(n, d):
    """Class id of every grid point, shape [N]."""
    idx = np.arange(n ** d)
    c = np.zeros(n ** d, dtype=np.int64)
    for a in range(d):
        ia = (idx // n ** a) % n
        ca = np.where(ia == 0, LO, np.where(ia == n - 1, HI, MID))
        c += ca * 3 ** a
    return c
