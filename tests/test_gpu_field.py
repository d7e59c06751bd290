"""The scattered field away from the grid and its far-field pattern on the
GPU (lsp_exterior_field, lsp_far_field) against the oracle (oracle/field.py)
evaluated on the same u: receivers on a circle / sphere around the domain,
points inside the domain and exactly on grid points (where the self term
applies), 1e-12 relative; at the grid points the field is the solution
itself (the discrete equation, to its solve tolerance); more than 16
right-hand sides (two launches) give each right-hand side its own result.
"""
import numpy as np
import pytest

import synth
from oracle.field import exterior_field, far_field

pytestmark = pytest.mark.gpu


def _lsp():
    import torch
    from paper_1408_4495_amd import lsp
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lsp.load()
    return lsp, torch


def _sphere(count, d, radius, centre=0.5):
    if d == 2:
        th = 2 * np.pi * np.arange(count) / count
        return centre + radius * np.stack([np.cos(th), np.sin(th)], axis=1)
    return centre + radius * synth.directions_fibonacci(count)


def _solve(lsp, n, d, m, dirs, omega):
    plan = lsp.Plan(n, d, max_nrhs=len(dirs), tol=1e-10)
    pb = lsp.Problem(plan, omega, m)
    pb.factor()
    uI = synth.plane_waves(n, d, omega, dirs)
    u, info, st = pb.solve(uI)
    assert st == 0
    return pb, uI, u


@pytest.mark.parametrize("d", [2, 3])
def test_field_matches_oracle(d):
    lsp, torch = _lsp()
    n = 32 if d == 2 else 16
    omega = 2 * np.pi * n / 8.0
    rng = np.random.default_rng([11, d])
    m = synth.medium_bumps(n, d, rng, 3, 0.3, 0.7, 0.06, 0.12, 0.1, 0.3)
    dirs = synth.directions_2d(3) if d == 2 else synth.directions_fibonacci(3)
    pb, uI, u = _solve(lsp, n, d, m, dirs, omega)
    un = u.cpu().numpy()
    X = synth.grid_coords(n, d)
    pts = np.concatenate([_sphere(40, d, 1.5), rng.uniform(0.05, 0.95, (20, d)), X[rng.integers(0, n ** d, 10)]])
    v = pb.exterior_field(u, uI, pts).cpu().numpy()
    ref = exterior_field(n, d, omega, m, un, uI, pts)
    assert np.max(np.abs(v - ref)) <= 1e-12 * np.max(np.abs(ref))
    xh = _sphere(33, d, 1.0, 0.0)
    A = pb.far_field(u, uI, xh).cpu().numpy()
    Aref = far_field(n, d, omega, m, un, uI, xh)
    assert np.max(np.abs(A - Aref)) <= 1e-12 * np.max(np.abs(Aref))
    # at every grid point the representation is the discrete equation: u itself
    g = pb.exterior_field(u, uI, X).cpu().numpy()
    assert np.linalg.norm(g - un) <= 1e-8 * np.linalg.norm(un)


def test_field_many_rhs_grouping():
    """18 right-hand sides (a group of 16 and one of 2) equal the solo
    evaluations bit for bit."""
    lsp, torch = _lsp()
    n, d = 16, 2
    omega = 2 * np.pi * 2
    m = synth.medium_single_bump(n, d, 0.3, 0.12)
    pb, uI, u = _solve(lsp, n, d, m, synth.directions_2d(18), omega)
    pts = _sphere(70, d, 2.0)
    v = pb.exterior_field(u, uI, pts).cpu().numpy()
    A = pb.far_field(u, uI, _sphere(5, d, 1.0, 0.0)).cpu().numpy()
    for r in (0, 15, 17):
        vs = pb.exterior_field(u[r:r + 1], uI[r:r + 1], pts).cpu().numpy()
        As = pb.far_field(u[r:r + 1], uI[r:r + 1], _sphere(5, d, 1.0, 0.0)).cpu().numpy()
        assert np.array_equal(vs[0], v[r]) and np.array_equal(As[0], A[r])


def test_field_receivers_2d_n256():
    """The 2D n = 256 benchmark medium, 360 receivers at radius 1.5 and 360
    far-field directions against the oracle."""
    lsp, torch = _lsp()
    w = synth.workload("c2")
    n, d, omega, m = w["n"], w["d"], w["omega"], w["m"]
    plan = lsp.Plan(n, d)
    pb = lsp.Problem(plan, omega, m)
    pb.factor()
    u, info, st = pb.solve(w["uI"])
    un = u.cpu().numpy()
    pts = _sphere(360, d, 1.5)
    v = pb.exterior_field(u, w["uI"], pts).cpu().numpy()
    ref = exterior_field(n, d, omega, m, un, w["uI"], pts)
    assert np.max(np.abs(v - ref)) <= 1e-12 * np.max(np.abs(ref))
    xh = _sphere(360, d, 1.0, 0.0)
    A = pb.far_field(u, w["uI"], xh).cpu().numpy()
    assert np.max(np.abs(A - far_field(n, d, omega, m, un, w["uI"], xh))) <= 1e-12 * np.max(np.abs(A))
