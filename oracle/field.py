"""The scattered field away from the grid (oracle; test infrastructure).

Section 1: once u is known on Omega, the scattered field everywhere is
  u(x) = - int_Omega G(x - y) w^2 m(y) (u(y) + u_I(y)) dy,
and it satisfies the radiation condition by construction.  With the grid
quadrature of Section 2.1 (weights h^d, and k_0 at a coincident grid point):
  u(x) = - sum_j h^d G(x - x_j) w^2 m_j (u_j + u_I,j)     (x != every x_j),
  u(x_i) = - sum_j k_{i-j} w^2 m_j (u_j + u_I,j)           (x = x_i),
so at the grid points it returns the discrete equation's own solution.
Far away, G(x - y) = c_d e^{i w |x|} |x|^{-(d-1)/2} e^{-i w xhat.y} (1 + O(1/|x|))
with c_2 = e^{i pi/4} / sqrt(8 pi w) (the large-argument form of (i/4) H0)
and c_3 = 1 / (4 pi); the far-field pattern is the coefficient
  A(xhat) = - c_d sum_j h^d e^{-i w xhat.x_j} w^2 m_j (u_j + u_I,j),
u(x) = A(xhat) e^{i w |x|} |x|^{-(d-1)/2} + O(|x|^{-(d+1)/2}).
Plain loops over the points (numpy over the grid), complex128.
"""
import numpy as np
import scipy.special as sp

from .greens import self_term


def _coords(n, d):
    idx = np.arange(n ** d)
    return (np.stack([(idx // n ** a) % n for a in range(d)], axis=1) + 0.5) / n


def source_density(omega, m, u, uI):
    """w^2 m (u + u_I), shape [nrhs, N]."""
    return omega ** 2 * np.asarray(m)[None, :] * (np.atleast_2d(u) + np.atleast_2d(uI))


def exterior_field(n, d, omega, m, u, uI, points, self_term_mode=0):
    """u at arbitrary points ([P, d]) for each right-hand side: [nrhs, P]."""
    h = 1.0 / n
    X = _coords(n, d)
    q = source_density(omega, m, u, uI)
    k0 = self_term(h, omega, d, self_term_mode)
    out = np.zeros((q.shape[0], len(points)), dtype=np.complex128)
    for p, x in enumerate(np.atleast_2d(points)):
        r = np.sqrt(np.sum((X - x) ** 2, axis=1))
        w = np.empty(r.size, dtype=np.complex128)
        hit = r == 0.0
        rr = r[~hit]
        if d == 2:
            w[~hit] = h * h * 0.25j * sp.hankel1(0, omega * rr)
        else:
            w[~hit] = h ** 3 * np.exp(1j * omega * rr) / (4.0 * np.pi * rr)
        w[hit] = k0
        out[:, p] = -(q @ w)
    return out


def far_field_constant(omega, d):
    return np.exp(0.25j * np.pi) / np.sqrt(8.0 * np.pi * omega) if d == 2 else 1.0 / (4.0 * np.pi)


def far_field(n, d, omega, m, u, uI, dirs):
    """A(xhat) for unit directions dirs ([P, d]): [nrhs, P]."""
    h = 1.0 / n
    X = _coords(n, d)
    q = source_density(omega, m, u, uI)
    dirs = np.atleast_2d(np.asarray(dirs, dtype=np.float64))
    E = np.exp(-1j * omega * (X @ dirs.T)) * h ** d   # [N, P]
    return -far_field_constant(omega, d) * (q @ E)
