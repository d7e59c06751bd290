"""Green's function, kernel table and self-term (oracle; test infrastructure).

Section 1 gives the free-space Green's function of -(Laplacian + w^2):
  d = 2: G(x) = (i/4) H0^(1)(w |x|),   d = 3: G(x) = exp(i w |x|) / (4 pi |x|).
Section 2.1 discretises the convolution with the trapezoid rule on the grid:
  k_t = G(h t) h^d for t != 0; k_0 is a local quadrature correction whose
  value the paper does not print.  Reading used here: k_0 is the exact
  integral of G over the disk (2D) / ball (3D) whose area / volume equals
  one grid cell h^d, i.e. radius rho = h/sqrt(pi) (2D), h (3/(4 pi))^(1/3) (3D).
  Closed forms (from d/dz[z H1(z)] = z H0(z), lim_{z->0} z H1^(1)(z) = -2i/pi,
  and the antiderivative of r exp(i w r)):
    2D: k_0 = (i pi rho / (2 w)) H1^(1)(w rho) - 1/w^2
    3D: k_0 = (exp(i w rho)(1 - i w rho) - 1) / w^2
  A second option (self_term 1) is the integral of G over the cell itself,
  computed here by plain adaptive quadrature of that definition.
  A third (self_term 2) is a one-point correction of the trapezoid rule
  fitted to a smooth probe: with g(x) = exp(-|x|^2 / (2 sigma^2)), g(0) = 1,
    k_0 = int G g dx - sum_{t != 0} h^d G(h t) g(h t),
  so that the corrected rule integrates G g exactly.  The trapezoid rule's
  error on G f for smooth f has a leading local term proportional to f(0)
  (Section 2.1: a one-point correction of order h^4 log(1/h)); k_0 fitted
  on g carries that term plus O(h^4 / sigma^2), so the discrete
  convolution converges at fourth order where the disk / ball term gives
  second.  sigma = max(0.05, 3h) (fixed in the domain's units, at least
  three grid steps so that the trapezoid rule resolves g).

Section 5 (eq:lap, eq:lslap): the 3D Laplace equation with a potential V is
the limit w -> 0: G(x) = 1/(4 pi |x|), and the ball self-term tends to
rho^2 / 2 (the series of exp(i w rho)(1 - i w rho) - 1 starts at (w rho)^2 / 2).
omega = 0 selects it (3D only; the paper treats no 2D Laplace case).
"""
import numpy as np
import scipy.special as sp


def green(r, omega, d):
    """G at distance r > 0 (Section 1; omega = 0: Section 5's 1/(4 pi r))."""
    r = np.asarray(r, dtype=np.float64)
    if d == 2:
        if omega == 0:
            raise ValueError("the Laplace case (omega = 0) is three-dimensional")
        return 0.25j * sp.hankel1(0, omega * r)
    if d == 3:
        return np.exp(1j * omega * r) / (4.0 * np.pi * r)
    raise ValueError("d must be 2 or 3")


def self_radius(h, d):
    """Radius of the disk/ball with the area/volume of one cell."""
    if d == 2:
        return h / np.sqrt(np.pi)
    return h * (3.0 / (4.0 * np.pi)) ** (1.0 / 3.0)


def self_term(h, omega, d, mode=0):
    """k_0 (Section 2.1's local correction; its value is not printed).
    mode 0: integral of G over the equal-measure disk/ball (reading above);
    mode 1: integral of G over the grid cell [-h/2, h/2]^d itself;
    mode 2: the one-point correction fitted to a Gaussian probe."""
    if mode == 1:
        return cell_self_term(h, omega, d)
    if mode == 2:
        return fitted_self_term(h, omega, d)
    rho = self_radius(h, d)
    if d == 2:
        if omega == 0:
            raise ValueError("the Laplace case (omega = 0) is three-dimensional")
        return 1j * np.pi * rho / (2.0 * omega) * sp.hankel1(1, omega * rho) - 1.0 / omega ** 2
    if omega == 0:
        return complex(rho * rho / 2.0)  # integral of 1/(4 pi r) over the ball
    return (np.exp(1j * omega * rho) * (1.0 - 1j * omega * rho) - 1.0) / omega ** 2


def cell_self_term(h, omega, d):
    """Integral of G over the cell [-h/2, h/2]^d, by adaptive Cartesian
    quadrature over the positive quadrant / octant (G is even in every axis),
    real and imaginary parts separately; the singularity of G sits at the
    integration region's corner."""
    from scipy import integrate
    a = 0.5 * h
    if d == 2:
        def part(fn):
            val, _ = integrate.dblquad(lambda y, x: fn(green(np.hypot(x, y), omega, 2)), 0.0, a, 0.0, a,
                                       epsabs=1e-16 * h * h, epsrel=1e-12)
            return val
        return 4.0 * (part(np.real) + 1j * part(np.imag))

    def part3(fn):
        val, _ = integrate.tplquad(lambda z, y, x: fn(green(np.sqrt(x * x + y * y + z * z), omega, 3)),
                                   0.0, a, 0.0, a, 0.0, a, epsabs=1e-16 * h * h, epsrel=1e-11)
        return val
    return 8.0 * (part3(np.real) + 1j * part3(np.imag))


def fitted_sigma(h):
    return max(0.05, 3.0 * h)


def gaussian_integral(omega, d, sigma):
    """int over R^d of G(x) exp(-|x|^2 / (2 sigma^2)) dx, in closed form:
    2D from int_0^inf J0(w r) e^{-a r^2} r dr = e^{-x} / (2a) and
    int_0^inf Y0(w r) e^{-a r^2} r dr = e^{-x} Ei(x) / (2 pi a), x = w^2 / (4a);
    3D from int_0^inf r e^{i w r - a r^2} dr = 1/(2a) + (i w / (2a))
    (sqrt(pi) e^{-z^2} / (2 sqrt(a)) + i F(z) / sqrt(a)), z = w / (2 sqrt(a)),
    F Dawson's integral; a = 1 / (2 sigma^2)."""
    a = 0.5 / (sigma * sigma)
    if d == 2:
        import mpmath
        x = omega * omega / (4.0 * a)
        with mpmath.workdps(40):  # e^{-x} Ei(x) without overflow for large x
            ex = float(mpmath.exp(-mpmath.mpf(x)) * mpmath.ei(mpmath.mpf(x)))
        J = np.exp(-x) / (2.0 * a)
        Y = ex / (2.0 * np.pi * a)
        return complex(-0.5 * np.pi * Y, 0.5 * np.pi * J)  # 2 pi (i/4) (J + i Y)
    z = omega / (2.0 * np.sqrt(a))
    I0 = np.sqrt(np.pi) / (2.0 * np.sqrt(a)) * np.exp(-z * z) + 1j * sp.dawsn(z) / np.sqrt(a)
    return complex(1.0 / (2.0 * a) + 1j * omega / (2.0 * a) * I0)


def fitted_self_term(h, omega, d, sigma=None):
    """k_0 = int G g - sum_{t != 0} h^d G(h t) g(h t), g a unit Gaussian of
    width sigma: the integral in closed form (gaussian_integral), the
    lattice sum over every t with 0 < |t| h <= 12 sigma (beyond it
    g < 1e-31)."""
    sigma = fitted_sigma(h) if sigma is None else sigma
    if d == 2 and omega == 0:
        raise ValueError("the Laplace case (omega = 0) is three-dimensional")
    a = 0.5 / (sigma * sigma)
    R = 12.0 * sigma
    m = int(np.floor(R / h))
    t = np.arange(-m, m + 1, dtype=np.float64)
    T = np.meshgrid(*([t] * d), indexing="ij")
    r = h * np.sqrt(sum(x * x for x in T))
    keep = (r > 0) & (r <= R)
    lattice = np.sum(green(r[keep], omega, d) * np.exp(-a * r[keep] ** 2)) * h ** d
    return complex(gaussian_integral(omega, d, sigma) - lattice)


def kernel_table(n, d, omega, self_term_mode=0):
    """k_t for t in [0, n]^d (absolute offsets per axis), shape (n+1,)*d.

    k depends on |t| only, so the table is symmetric under any permutation
    of its axes and covers every offset -n <= t_a <= n by reflection."""
    h = 1.0 / n
    ax = np.arange(n + 1, dtype=np.float64)
    T = np.meshgrid(*([ax] * d), indexing="ij")
    r = h * np.sqrt(sum(t * t for t in T))
    k = np.empty(r.shape, dtype=np.complex128)
    nz = r > 0
    k[nz] = green(r[nz], omega, d) * h ** d
    k[(0,) * d] = self_term(h, omega, d, self_term_mode)
    return k
