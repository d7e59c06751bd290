"""The discrete Lippmann-Schwinger operator (oracle; test infrastructure).

eq:lsd / eq:lso: (I + K w^2 m) u = g with K(i, j) = k_{i-j} over the n^d grid.
The right-hand side (eq:ls) discretised by the same quadrature is
g = K(-w^2 m u_I).  Fields are vectors of length N = n^d with linear index
l = i1 + n i2 (+ n^2 i3); reshaped to (n,)*d the array axes run (i_d..i_1).

Three tiers of K v:
  dense_K      -- the N x N matrix itself (N <= a few thousand),
  apply_K_direct -- O(N^2) direct summation, blocked over rows,
  apply_K_fft  -- circulant embedding on (2n)^d and numpy FFTs (Section 1
                  notes the convolution structure allows FFT application).
"""
import numpy as np

from .greens import kernel_table


def grid_index(n, d):
    """Integer multi-index of every grid point, shape [N, d], column a = i_{a+1}."""
    idx = np.arange(n ** d)
    return np.stack([(idx // n ** a) % n for a in range(d)], axis=1)


def dense_K(n, d, omega, ktab=None):
    if ktab is None:
        ktab = kernel_table(n, d, omega)
    I = grid_index(n, d)
    T = np.abs(I[:, None, :] - I[None, :, :])
    return ktab[tuple(T[..., a] for a in range(d))]


def apply_K_direct(v, n, d, omega, ktab=None, block=256):
    """y_i = sum_j k_{i-j} v_j by direct summation; v shape [N] or [nrhs, N]."""
    if ktab is None:
        ktab = kernel_table(n, d, omega)
    v = np.asarray(v, dtype=np.complex128)
    single = v.ndim == 1
    V = v[None, :] if single else v
    I = grid_index(n, d)
    Y = np.zeros_like(V)
    for r0 in range(0, I.shape[0], block):
        T = np.abs(I[r0:r0 + block, None, :] - I[None, :, :])
        Kb = ktab[tuple(T[..., a] for a in range(d))]
        Y[:, r0:r0 + block] = V @ Kb.T
    return Y[0] if single else Y


def embedded_kernel(n, d, omega, ktab=None):
    """Kernel on the (2n)^d periodic grid: entry at wrapped offset t holds
    k_t for |t_a| < n on every axis, zero where some |t_a| = n."""
    if ktab is None:
        ktab = kernel_table(n, d, omega)
    L = 2 * n
    t = np.arange(L)
    off = np.where(t < n, t, L - t)          # |wrapped offset|
    valid = t != n
    idx = np.meshgrid(*([off] * d), indexing="ij")
    kk = ktab[tuple(idx)]
    mask = np.ones((L,) * d, dtype=bool)
    for a in range(d):
        shape = [1] * d
        shape[a] = L
        mask &= valid.reshape(shape)
    return np.where(mask, kk, 0.0)


def apply_K_fft(v, n, d, omega, khat=None):
    """K v by zero-padded FFT convolution on the (2n)^d circulant embedding."""
    if khat is None:
        khat = np.fft.fftn(embedded_kernel(n, d, omega))
    v = np.asarray(v, dtype=np.complex128)
    single = v.ndim == 1
    V = v[None, :] if single else v
    L = 2 * n
    Y = np.empty_like(V)
    for r in range(V.shape[0]):
        pad = np.zeros((L,) * d, dtype=np.complex128)
        pad[(slice(0, n),) * d] = V[r].reshape((n,) * d)
        conv = np.fft.ifftn(np.fft.fftn(pad) * khat)
        Y[r] = conv[(slice(0, n),) * d].reshape(-1)
    return Y[0] if single else Y


class Operator:
    """A = I + K p and g = K(-p u_I) with p = w^2 m, or for Section 5's
    Laplace case (eq:lslap) p = V and g = K f; K applied by FFT."""

    def __init__(self, n, d, omega, m, ktab=None, potential=None):
        self.n, self.d, self.omega = n, d, float(omega)
        self.m = np.asarray(m, dtype=np.float64) if m is not None else None
        self.p = (np.asarray(potential, dtype=np.float64) if potential is not None
                  else self.omega ** 2 * self.m)
        self.ktab = kernel_table(n, d, omega) if ktab is None else ktab
        self.khat = np.fft.fftn(embedded_kernel(n, d, omega, self.ktab))

    def K(self, v):
        return apply_K_fft(v, self.n, self.d, self.omega, self.khat)

    def apply(self, u):
        return u + self.K(self.p * u)

    def rhs(self, uI):
        return self.K(-self.p * uI)

    def rhs_source(self, f):
        """g = K f: the source term of eq:lslap (G * f)."""
        return self.K(np.asarray(f, dtype=np.complex128))
