"""Pins of the general-domain oracle (Section 4) against what the method and
the mathematics fix, independent of the oracle's own code paths:

  * the boundary set and neighbourhoods against brute-force loops;
  * the sketch with R = identity on Omega reproduces the exact local
    problem min ||alpha (K w^2 m)(mu(i), Omega)|| solved from the dense K;
  * a rank-one medium (one nonzero of m) is annihilated exactly by every
    boundary row, so those rows of Q(I + K w^2 m) - M vanish;
  * each boundary alpha is optimal for its sketch (no unit vector better);
  * Omega = the whole box: the interior rows are the rectangle's and the
    solution is the rectangle oracle's;
  * the solution equals a dense solve of the restricted system;
  * the preconditioner cuts GMRES iterations several-fold on the paper's
    smoothed l2 / l1 cavities (its qualitative claim for near-convex Omega).
"""
import numpy as np
import pytest

import synth
from oracle.general import GeneralProblem, classify, neighbour_offsets, boundary_stencil
from oracle.operator import dense_K
from oracle.solve import OracleProblem
from oracle.gmres import gmres


def test_general_classification_brute_force():
    n, d = 9, 2
    mask = synth.domain_mask(n, d, "l2", radius=0.4)
    pts, nb, interior = classify(mask, n, d)
    M = mask.reshape(n, n)  # [i2, i1]
    assert np.array_equal(pts, np.nonzero(mask)[0])
    for k, p in enumerate(pts):
        i1, i2 = p % n, p // n
        inner = True
        for s2 in (-1, 0, 1):
            for s1 in (-1, 0, 1):
                j1, j2 = i1 + s1, i2 + s2
                q = (s1 + 1) + 3 * (s2 + 1)
                ok = 0 <= j1 < n and 0 <= j2 < n and M[j2, j1]
                assert nb[k, q] == (j1 + n * j2 if ok else -1)
                inner = inner and ok
        assert interior[k] == inner
    assert 0 < np.sum(~interior) < pts.size


def _gp(n, d, m, mask, R, omega=None):
    omega = 2 * np.pi * n / 8.0 if omega is None else omega
    return GeneralProblem(n, d, omega, m, mask, R)


def test_general_identity_sketch_is_the_exact_local_problem():
    """With R = the identity on Omega (r = |Omega|), T = (K w^2 m)(:, Omega)
    exactly; each boundary alpha must be the minimiser of the full local
    matrix built from the dense K (up to its phase convention)."""
    n, d = 12, 2
    mask = synth.domain_mask(n, d, "l2")
    m = synth.medium_cavity(n, d, "l2")
    pts = np.nonzero(mask)[0]
    R = np.zeros((pts.size, n ** d))
    R[np.arange(pts.size), pts] = 1.0
    g = _gp(n, d, m, mask, R)
    Kd = dense_K(n, d, g.omega, g.ktab)
    p = g.omega ** 2 * m
    checked = 0
    for k, i in enumerate(g.gst.points):
        sl = g.gst.slots[k]
        mu = i + np.array([s[0] + n * s[1] for s in neighbour_offsets(d)[sl]])
        X = Kd[np.ix_(mu, pts)] * p[pts][None, :]
        U, sig, _ = np.linalg.svd(X, full_matrices=False)
        np.testing.assert_allclose(g.gst.sigma[k], sig, rtol=1e-10, atol=1e-14 * sig[0])
        if sig[-2] - sig[-1] < 1e-3 * sig[0]:
            continue  # nearly degenerate least singular value: alpha not unique
        a = np.conj(U[:, -1])
        c = int(np.nonzero(sl == 4)[0][0])
        a = a / (a[c] / abs(a[c]))
        np.testing.assert_allclose(g.gst.alpha[k, sl], a, atol=1e-9)
        checked += 1
    assert checked > len(g.gst.points) // 2


def test_general_rank_one_medium_is_annihilated():
    """m nonzero at one point j: (K w^2 m)(mu(i), Omega) = K(mu(i), j) w^2 m_j
    has rank one, so alpha K(mu(i), j) = 0 and the boundary rows of
    E = Q (I + K w^2 m) - M vanish (interior rows keep their own residual)."""
    n, d = 16, 2
    mask = synth.domain_mask(n, d, "l2")
    m = np.zeros(n ** d)
    j = (n // 2) + n * (n // 2)
    m[j] = 0.3
    R = synth.sketch_matrix(n, d, 18, 77)
    g = _gp(n, d, m, mask, R)
    pts = g.pts
    Kd = dense_K(n, d, g.omega, g.ktab)[np.ix_(pts, pts)]
    A = np.eye(pts.size) + Kd * (g.omega ** 2 * m[pts])[None, :]
    E = g.Q.toarray() @ A - g.M.toarray()
    pos = np.searchsorted(pts, g.gst.points)
    scale = np.abs(Kd).max() * g.omega ** 2 * 0.3
    assert np.max(np.abs(E[pos])) <= 1e-12 * scale
    # the interior rows are the rectangle's and do not vanish in general
    assert np.max(np.abs(np.delete(E, pos, axis=0))) > 1e-6 * scale


def test_general_boundary_alpha_is_optimal():
    w = synth.workload("g1")
    g = _gp(w["n"], w["d"], w["m"], w["mask"], w["R"], w["omega"])
    rng = np.random.default_rng(5)
    for k, i in enumerate(g.gst.points[::7]):
        kk = k * 7
        sl = g.gst.slots[kk]
        mu = g.nb[np.searchsorted(g.pts, g.gst.points[kk]), sl]
        X = g.T[:, mu].T
        a = g.gst.alpha[kk, sl]
        assert abs(np.linalg.norm(a) - 1) < 1e-13
        val = np.linalg.norm(a @ X)
        assert abs(val - g.gst.sigma[kk][-1]) <= 1e-10 * g.gst.sigma[kk][0]
        for _ in range(20):
            v = rng.standard_normal(sl.size) + 1j * rng.standard_normal(sl.size)
            v /= np.linalg.norm(v)
            assert np.linalg.norm(v @ X) >= val * (1 - 1e-12)
            pert = a + 1e-3 * v
            pert /= np.linalg.norm(pert)
            assert np.linalg.norm(pert @ X) >= val * (1 - 1e-12)
    # and the helper is the SVD's least left singular vector
    X = rng.standard_normal((5, 9)) + 1j * rng.standard_normal((5, 9))
    a, sig = boundary_stencil(X)
    assert abs(np.linalg.norm(a @ X) - sig[-1]) < 1e-12


def test_general_full_box_reduces_to_the_rectangle():
    n, d = 16, 2
    omega = 2 * np.pi * 2
    m = synth.medium_single_bump(n, d, 0.2, 0.12)
    mask = np.ones(n ** d, dtype=bool)
    R = synth.sketch_matrix(n, d, 18, 78)
    g = _gp(n, d, m, mask, R, omega)
    rect = OracleProblem(n, d, omega, m)
    cls_outer = np.array([(p % n) in (0, n - 1) or (p // n) in (0, n - 1) for p in range(n * n)])
    assert np.array_equal(np.sort(g.gst.points), np.nonzero(cls_outer)[0])
    ip = np.nonzero(~cls_outer)[0]
    Mg, Mr = g.M.toarray(), rect.M.toarray()
    np.testing.assert_allclose(Mg[ip], Mr[ip], rtol=0, atol=1e-14 * np.abs(Mr).max())
    uI = synth.plane_waves(n, d, omega, [[0.0, -1.0]])[0]
    ug = g.solve(uI, tol=1e-12).x
    ur = rect.solve(uI, tol=1e-12).x
    assert np.linalg.norm(ug - ur) <= 1e-10 * np.linalg.norm(ur)


@pytest.mark.parametrize("kind", ["l2", "l1"])
def test_general_solution_matches_dense_solve(kind):
    n, d = 16, 2
    omega = 2 * np.pi * n / 8.0
    mask = synth.domain_mask(n, d, kind)
    m = synth.medium_cavity(n, d, kind)
    g = _gp(n, d, m, mask, synth.sketch_matrix(n, d, 18, 79), omega)
    uI = synth.plane_waves(n, d, omega, [[0.0, -1.0]])[0]
    res = g.solve(uI)
    pts = g.pts
    Kd = dense_K(n, d, omega, g.ktab)
    p = omega ** 2 * m
    A = np.eye(pts.size) + Kd[np.ix_(pts, pts)] * p[pts][None, :]
    rhs = -(Kd[pts][:, pts] @ (p[pts] * uI[pts]))
    u = np.linalg.solve(A, rhs)
    assert res.converged and res.relres <= 1e-8
    assert np.linalg.norm(res.x - u) <= 1e-7 * np.linalg.norm(u)


@pytest.mark.parametrize("kind", ["l2", "l1"])
def test_general_preconditioner_cuts_iterations(kind):
    n, d = 64, 2
    omega = 2 * np.pi * n / 8.0
    mask = synth.domain_mask(n, d, kind)
    m = synth.medium_cavity(n, d, kind)
    g = _gp(n, d, m, mask, synth.sketch_matrix(n, d, 18, 80), omega)
    uI = synth.plane_waves(n, d, omega, [[0.0, -1.0]])[0]
    pre = g.solve(uI)
    plain = gmres(g.apply, lambda v: v, g.rhs(uI), 1e-8, 30, 400)
    assert pre.converged and pre.iters <= 15, pre.iters
    assert plain.iters >= 3 * pre.iters, (plain.iters, pre.iters)
