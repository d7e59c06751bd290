"""Pins of the scattered-field evaluation oracle (Section 1's representation
of u outside Omega) against facts fixed by the mathematics:

  * at the grid points the representation returns the discrete equation's
    own solution (the Lippmann-Schwinger equation itself);
  * far away the field equals A(xhat) e^{i w r} r^{-(d-1)/2} (checked against
    scipy's Hankel function at a large radius, independent of the
    far-field constants);
  * reciprocity of the discrete problem (symmetric kernel table):
    A(xhat; dhat) = A(-dhat; -xhat);
  * a one-point medium (a Foldy point scatterer) has the closed-form far
    field -c_d h^d w^2 m_j u_I(x_j) e^{-i w xhat.x_j} / (1 + k_0 w^2 m_j).
"""
import numpy as np
import pytest

import synth
from oracle.field import exterior_field, far_field, far_field_constant
from oracle.greens import self_term
from oracle.solve import OracleProblem


def _problem(n, d, omega, m, dirs, tol=1e-12):
    prob = OracleProblem(n, d, omega, m)
    uI = synth.plane_waves(n, d, omega, dirs)
    u = np.stack([prob.solve(uI[r], tol=tol).x for r in range(uI.shape[0])])
    return prob, uI, u


@pytest.mark.parametrize("d", [2, 3])
def test_field_at_grid_points_is_the_solution(d):
    n = 16 if d == 2 else 8
    omega = 2 * np.pi * n / 8.0
    m = synth.medium_single_bump(n, d, 0.3, 0.15)
    dirs = [[1.0, 0.0]] if d == 2 else [[0.0, 0.0, -1.0]]
    prob, uI, u = _problem(n, d, omega, m, dirs)
    X = synth.grid_coords(n, d)
    v = exterior_field(n, d, omega, m, u, uI, X)
    assert np.linalg.norm(v - u) <= 1e-9 * np.linalg.norm(u)


@pytest.mark.parametrize("d", [2, 3])
def test_far_field_is_the_large_radius_limit(d):
    n = 16 if d == 2 else 8
    omega = 2 * np.pi * n / 8.0
    m = synth.medium_single_bump(n, d, 0.3, 0.15)
    dirs = [[0.6, 0.8]] if d == 2 else [[0.0, 0.6, 0.8]]
    prob, uI, u = _problem(n, d, omega, m, dirs)
    rng = np.random.default_rng(3)
    xh = rng.standard_normal((5, d))
    xh /= np.linalg.norm(xh, axis=1, keepdims=True)
    R = 1e8
    uf = exterior_field(n, d, omega, m, u, uI, R * xh)
    A = far_field(n, d, omega, m, u, uI, xh)
    lim = uf * R ** ((d - 1) / 2.0) * np.exp(-1j * omega * R)
    assert np.max(np.abs(lim - A)) <= 5e-6 * np.max(np.abs(A))
    # the constant alone would not do: a wrong sign of the phase fails
    Aw = far_field(n, d, omega, m, u, uI, -xh)
    assert np.max(np.abs(lim - Aw)) > 1e-2 * np.max(np.abs(A))


@pytest.mark.parametrize("d", [2, 3])
def test_far_field_reciprocity(d):
    n = 16 if d == 2 else 8
    omega = 2 * np.pi * n / 8.0
    rng = np.random.default_rng([7, d])
    m = synth.medium_bumps(n, d, rng, 3, 0.3, 0.7, 0.08, 0.15, 0.1, 0.4)
    a = rng.standard_normal(d)
    b = rng.standard_normal(d)
    a /= np.linalg.norm(a)
    b /= np.linalg.norm(b)
    # incident dhat = a observed at xhat = b, against incident -b observed at -a
    prob, uI, u = _problem(n, d, omega, m, [a, -b])
    A_ab = far_field(n, d, omega, m, u[0], uI[0], [b])[0, 0]
    A_ba = far_field(n, d, omega, m, u[1], uI[1], [-a])[0, 0]
    assert abs(A_ab - A_ba) <= 1e-9 * abs(A_ab)
    assert abs(A_ab) > 1e-6


@pytest.mark.parametrize("d", [2, 3])
def test_point_scatterer_closed_form(d):
    n = 16 if d == 2 else 8
    omega = 2 * np.pi * n / 8.0
    h = 1.0 / n
    m = np.zeros(n ** d)
    j = 5 + n * 7 + (n * n * 3 if d == 3 else 0)
    m[j] = 0.4
    dirs = [[1.0, 0.0]] if d == 2 else [[0.0, 0.0, 1.0]]
    prob, uI, u = _problem(n, d, omega, m, dirs)
    xh = np.array([[0.0, 1.0]] if d == 2 else [[1.0, 0.0, 0.0]])
    A = far_field(n, d, omega, m, u, uI, xh)[0, 0]
    k0 = self_term(h, omega, d)
    w2m = omega ** 2 * 0.4
    xj = synth.grid_coords(n, d)[j]
    ref = -far_field_constant(omega, d) * h ** d * w2m * uI[0, j] * np.exp(-1j * omega * xh[0] @ xj) / (1 + k0 * w2m)
    assert abs(A - ref) <= 1e-10 * abs(ref)
