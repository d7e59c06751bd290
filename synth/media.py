"""Seeded media, incident fields and test vectors (see package docstring).

Seeds: numpy.random.default_rng([14084495, k]) for workload k, draws taken in
the order each generator lists them.
"""
import math
import numpy as np

SEED_BASE = 14084495


def grid_coords(n, d):
    """Cell-centred coordinates, shape [n^d, d], linear index i1 fastest."""
    ax = (np.arange(n, dtype=np.float64) + 0.5) / n
    mesh = np.meshgrid(*([ax] * d), indexing="ij")
    # meshgrid 'ij' puts axis 0 slowest; reverse so that i1 (axis 0 of x) is fastest
    cols = [mesh[a].transpose(tuple(range(d))[::-1]).reshape(-1) for a in range(d)]
    return np.stack(cols, axis=1)


def medium_single_bump(n, d, amp=0.2, width=0.1, centre=None):
    """m(x) = amp * exp(-|x-c|^2 / (2 width^2)), c = (1/2, ..., 1/2) by default."""
    X = grid_coords(n, d)
    c = np.full(d, 0.5) if centre is None else np.asarray(centre, dtype=np.float64)
    r2 = np.sum((X - c) ** 2, axis=1)
    return amp * np.exp(-r2 / (2.0 * width * width))


def medium_bumps(n, d, rng, count, centre_lo, centre_hi, w_lo, w_hi, a_lo, a_hi):
    """Sum of `count` Gaussian bumps.  Draw order: centres (count x d),
    widths (count), amplitudes (count)."""
    c = rng.uniform(centre_lo, centre_hi, size=(count, d))
    w = rng.uniform(w_lo, w_hi, size=count)
    a = rng.uniform(a_lo, a_hi, size=count)
    X = grid_coords(n, d)
    m = np.zeros(X.shape[0])
    for k in range(count):
        r2 = np.sum((X - c[k]) ** 2, axis=1)
        m += a[k] * np.exp(-r2 / (2.0 * w[k] * w[k]))
    return m


def medium_disks(n, rng, count=40, c_lo=0.1, c_hi=0.9, r_lo=0.01, r_hi=0.05,
                 v_lo=0.0, v_hi=0.4):
    """`count` disks with tanh-smoothed edges (edge width 2h), combined by max.
    Draw order: centres (count x 2), radii (count), values (count)."""
    c = rng.uniform(c_lo, c_hi, size=(count, 2))
    r = rng.uniform(r_lo, r_hi, size=count)
    v = rng.uniform(v_lo, v_hi, size=count)
    X = grid_coords(n, 2)
    delta = 2.0 / n
    m = np.zeros(X.shape[0])
    for k in range(count):
        dist = np.sqrt(np.sum((X - c[k]) ** 2, axis=1))
        m = np.maximum(m, v[k] * 0.5 * (1.0 - np.tanh((dist - r[k]) / delta)))
    return m


def potential_gaussian(n, peak_h2=1.1, width=0.12, centre=None):
    """Section 5's first example: a negative Gaussian potential,
    V(x) = -peak_h2 n^2 exp(-|x - c|^2 / (2 width^2)), c = (1/2, 1/2, 1/2)
    (V proportional to 1/h^2 so that the problem loses ellipticity)."""
    X = grid_coords(n, 3)
    c = np.full(3, 0.5) if centre is None else np.asarray(centre, dtype=np.float64)
    r2 = np.sum((X - c) ** 2, axis=1)
    return -peak_h2 * n * n * np.exp(-r2 / (2.0 * width * width))


def potential_ball(n, peak_h2=1.1, radius=0.25, centre=None):
    """Section 5's second example: a negative smoothed characteristic
    function of a ball, V(x) = -peak_h2 n^2 (1 - tanh((|x - c| - radius) / (2h))) / 2."""
    X = grid_coords(n, 3)
    c = np.full(3, 0.5) if centre is None else np.asarray(centre, dtype=np.float64)
    dist = np.sqrt(np.sum((X - c) ** 2, axis=1))
    return -peak_h2 * n * n * 0.5 * (1.0 - np.tanh((dist - radius) * n / 2.0))


def delta_source(n, d, points):
    """Discrete delta sources: row k is e_j / h^d at the grid point j nearest
    to points[k] (so that the grid quadrature of f is 1)."""
    points = np.atleast_2d(np.asarray(points, dtype=np.float64))
    f = np.zeros((points.shape[0], n ** d), dtype=np.complex128)
    for k, x in enumerate(points):
        i = np.clip(np.floor(x * n).astype(np.int64), 0, n - 1)
        f[k, int(np.sum(i * n ** np.arange(d)))] = float(n) ** d
    return f


def cavity_rho(n, d, kind="l2", radius=0.45, centre=None):
    """Scaled distance |x - c|_p / radius of every grid point (p = 2 for the
    disk / ball, p = 1 for the diamond / octahedron, p = inf for the square /
    cube)."""
    X = grid_coords(n, d)
    c = np.full(d, 0.5) if centre is None else np.asarray(centre, dtype=np.float64)
    Y = X - c
    if kind == "l2":
        dist = np.sqrt(np.sum(Y * Y, axis=1))
    elif kind == "linf":
        dist = np.max(np.abs(Y), axis=1)
    else:
        dist = np.sum(np.abs(Y), axis=1)
    return dist / radius


def domain_mask(n, d, kind="l2", radius=0.45, centre=None):
    """The support Omega of a cavity medium: grid points with rho <= 1."""
    return cavity_rho(n, d, kind, radius, centre) <= 1.0


def medium_cavity(n, d, kind="l2", depth=-0.5, radius=0.45, core=0.6, centre=None):
    """Smoothed cavity of an l2, l1 or l-infinity ball: m = depth for rho <= core, a
    raised-cosine ramp to 0 at rho = 1, and 0 outside (support = the mask)."""
    rho = cavity_rho(n, d, kind, radius, centre)
    ramp = 0.5 * (1.0 + np.cos(np.pi * np.clip((rho - core) / (1.0 - core), 0.0, 1.0)))
    return depth * np.where(rho <= 1.0, ramp, 0.0)


def sketch_matrix(n, d, r, seed):
    """The r x n^d standard Gaussian matrix R of a general-domain set-up,
    rows = sketch columns (Section 4 draws it at random; seeded here)."""
    rng = np.random.default_rng([SEED_BASE, 2000 + int(seed)])
    return rng.standard_normal((r, n ** d))


def directions_2d(count, offset=0.0):
    """Unit vectors at angles offset + 2 pi j / count."""
    th = offset + 2.0 * np.pi * np.arange(count) / count
    return np.stack([np.cos(th), np.sin(th)], axis=1)


def random_rotation(rng):
    """Uniform random rotation from a normalised Gaussian quaternion."""
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def directions_fibonacci(count, rng=None):
    """Fibonacci-sphere directions z_k = 1-(2k+1)/count, phi_k = k*pi*(3-sqrt5),
    rotated by a seeded uniform rotation when rng is given."""
    k = np.arange(count)
    z = 1.0 - (2.0 * k + 1.0) / count
    phi = k * np.pi * (3.0 - math.sqrt(5.0))
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    D = np.stack([s * np.cos(phi), s * np.sin(phi), z], axis=1)
    if rng is not None:
        D = D @ random_rotation(rng).T
    return D


def plane_waves(n, d, omega, dirs):
    """u_I(x) = exp(i omega dhat.x) for each direction: shape [nrhs, n^d] complex128."""
    X = grid_coords(n, d)
    dirs = np.atleast_2d(np.asarray(dirs, dtype=np.float64))
    phase = omega * (dirs @ X.T)
    return np.exp(1j * phase)


def random_complex(shape, seed):
    """Standard complex Gaussian test vectors from a fixed seed."""
    rng = np.random.default_rng([SEED_BASE, 1000 + int(seed)])
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _c1():
    n, d = 32, 2
    omega = 2 * np.pi * 4
    m = medium_single_bump(n, d, 0.2, 0.1)
    uI = plane_waves(n, d, omega, [[1.0, 0.0]])
    return dict(name="2d_n32_single_bump", n=n, d=d, omega=omega, m=m, uI=uI)


def _c2():
    n, d = 256, 2
    omega = 2 * np.pi * 32
    rng = np.random.default_rng([SEED_BASE, 1])
    m = medium_bumps(n, d, rng, 8, 0.2, 0.8, 0.03, 0.08, 0.0, 0.3)
    th = rng.uniform(0.0, 2 * np.pi)
    uI = plane_waves(n, d, omega, [[np.cos(th), np.sin(th)]])
    return dict(name="2d_n256_8bumps", n=n, d=d, omega=omega, m=m, uI=uI)


def _c3():
    n, d = 1024, 2
    omega = 2 * np.pi * 128
    rng = np.random.default_rng([SEED_BASE, 2])
    m = medium_disks(n, rng)
    uI = plane_waves(n, d, omega, directions_2d(16))
    return dict(name="2d_n1024_40disks_16rhs", n=n, d=d, omega=omega, m=m, uI=uI)


def _c4():
    n, d = 64, 3
    omega = 2 * np.pi * 8
    rng = np.random.default_rng([SEED_BASE, 3])
    m = medium_bumps(n, d, rng, 6, 0.2, 0.8, 0.05, 0.12, 0.0, 0.3)
    uI = plane_waves(n, d, omega, directions_fibonacci(8, rng))
    return dict(name="3d_n64_6bumps_8rhs", n=n, d=d, omega=omega, m=m, uI=uI)


def _c4s():
    """The 3D recipe of the n=64 workload (same draws: bumps, rotation) on a
    32-point grid at 8 points per wavelength (omega = 8 pi)."""
    n, d = 32, 3
    omega = 2 * np.pi * 4
    rng = np.random.default_rng([SEED_BASE, 3])
    m = medium_bumps(n, d, rng, 6, 0.2, 0.8, 0.05, 0.12, 0.0, 0.3)
    uI = plane_waves(n, d, omega, directions_fibonacci(8, rng))
    return dict(name="3d_n32_6bumps_8rhs", n=n, d=d, omega=omega, m=m, uI=uI)


# Section 5's Laplace tests: a delta source near the top left corner of the
# middle cross-section (x1 = 1/8, x2 = 7/8, x3 = 1/2), potentials of about
# -1.1 / h^2 at their peak (the paper's 5.8e2, 2.3e3, 9.2e3 at N = 1.2e4, 1.0e5,
# 8.6e5); grids of 24, 48, 96 points per side.
LAPLACE_SOURCE = (0.125, 0.875, 0.5)


def _laplace(n, kind):
    V = potential_gaussian(n) if kind == "gauss" else potential_ball(n)
    f = delta_source(n, 3, [LAPLACE_SOURCE])
    return dict(name=f"3d_n{n}_laplace_{kind}", n=n, d=3, omega=0.0, m=None, V=V, f=f, laplace=True)


# Section 4's tests: smoothed cavities of an l2 ball and of an l1 ball
# (radius 0.45 around the centre, m = -0.5 in the core), a plane wave
# pointing down, 8 points per wavelength; the sketch has r = 2 * 3^d columns.
def _general(n, d, kind, seed):
    omega = 2 * np.pi * n / 8.0
    down = [0.0] * (d - 1) + [-1.0]
    r = 2 * 3 ** d
    return dict(name=f"{d}d_n{n}_{kind}_cavity", n=n, d=d, omega=omega, m=medium_cavity(n, d, kind),
                mask=domain_mask(n, d, kind), R=sketch_matrix(n, d, r, seed),
                uI=plane_waves(n, d, omega, [down]), general=True)


WORKLOADS = {"c1": _c1, "c2": _c2, "c3": _c3, "c4": _c4, "c4s": _c4s,
             "l1": lambda: _laplace(24, "gauss"), "l2": lambda: _laplace(48, "gauss"),
             "l3": lambda: _laplace(96, "gauss"), "l1b": lambda: _laplace(24, "ball"),
             "l2b": lambda: _laplace(48, "ball"),
             "g1": lambda: _general(32, 2, "l2", 1), "g1d": lambda: _general(32, 2, "l1", 2),
             "g2": lambda: _general(256, 2, "l2", 3), "g2d": lambda: _general(256, 2, "l1", 4),
             "g3": lambda: _general(32, 3, "l2", 5)}


def workload(key):
    """Return the seeded workload dict: Helmholtz (n, d, omega, m [N],
    uI [nrhs, N]) or Laplace (n, d = 3, omega = 0, V [N], f [nrhs, N])."""
    return WORKLOADS[key]()


def request_problem(n, d, nrhs, rng):
    """One serving request: 8-points-per-wavelength grid, Gaussian-bump medium,
    nrhs plane waves.  Draw order: medium, then direction offset/rotation."""
    omega = 2 * np.pi * n / 8.0
    if d == 2:
        m = medium_bumps(n, 2, rng, 8, 0.2, 0.8, 0.03, 0.08, 0.0, 0.3)
        dirs = directions_2d(nrhs, rng.uniform(0.0, 2 * np.pi))
    else:
        m = medium_bumps(n, 3, rng, 6, 0.2, 0.8, 0.05, 0.12, 0.0, 0.3)
        dirs = directions_fibonacci(nrhs, rng)
    return dict(n=n, d=d, omega=omega, m=m, uI=plane_waves(n, d, omega, dirs))


def serving_requests(count, rate_hz, seed=5, sizes=None, max_rhs=32):
    """Poisson stream of requests.  Draw order per request: exponential gap,
    size index, nrhs, then the request's own medium and directions."""
    rng = np.random.default_rng([SEED_BASE, 4, int(seed)])
    if sizes is None:
        sizes = [(128, 2), (256, 2), (512, 2), (32, 3), (48, 3)]
    t = 0.0
    out = []
    for k in range(count):
        t += rng.exponential(1.0 / rate_hz)
        n, d = sizes[int(rng.integers(len(sizes)))]
        nrhs = int(rng.integers(1, max_rhs + 1))
        prob = request_problem(n, d, nrhs, rng)
        prob["arrival"] = t
        prob["id"] = k
        out.append(prob)
    return out
