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
    mode 1: integral of G over the grid cell [-h/2, h/2]^d itself."""
    if mode == 1:
        return cell_self_term(h, omega, d)
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
