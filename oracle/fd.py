"""Finite-difference Laplacian and Hamiltonian on a periodic or Dirichlet grid (oracle).

Sec. 3 (Implementation): derivative operators are high-order centred finite
differences on a uniform real-space grid, integrals use the trapezoidal rule,
and the Hamiltonian is applied matrix-free.  Eq. 4 gives the Hamiltonian; for
the synthetic cells used here it reduces to H = -1/2 Lap_h + diag(V_loc)
(no exchange-correlation, no nonlocal part), with Lap_h the 12th-order
(radius-6) centred stencil applied along each axis.

Boundary conditions (bc): "periodic" (the synthetic crystals), or "dirichlet" (an isolated
system in a box, the real-space setting of Sec. 1): the grid points are x_i = (i + 1) h,
i = 0 .. n-1, the function vanishes outside, so every stencil reach beyond the grid reads 0.

Array convention: a grid function is a flat vector of length N_d with index
i = x + n0*(y + n1*z) (x fastest); as a NumPy array it is reshaped to
(n2, n1, n0) so that the last axis is x.  Blocks of vectors are arrays of
shape (N_d, nvec); batched grids are (B, n2, n1, n0).
"""
from fractions import Fraction
from math import factorial

import numpy as np

RADIUS = 6


def fd_weights_exact(radius=RADIUS):
    """Centred second-derivative weights w_0..w_M (M = radius) as exact rationals.

    The order-2M centred formula for f'' has w_p = 2(-1)^{p+1}(M!)^2 /
    (p^2 (M-p)! (M+p)!) for p >= 1 and w_0 = -2 sum_p w_p (so constants are
    annihilated).  Sec. 3 says only "high-order centred finite differences";
    the order (12, radius 6) is the one the workloads fix.
    """
    M = radius
    w = [Fraction(0)] * (M + 1)
    for p in range(1, M + 1):
        w[p] = Fraction(2 * (-1) ** (p + 1) * factorial(M) ** 2,
                        p * p * factorial(M - p) * factorial(M + p))
    w[0] = -2 * sum(w[1:])
    return w


def fd_weights(radius=RADIUS):
    return np.array([float(v) for v in fd_weights_exact(radius)])


def symbol_1d(theta, h, radius=RADIUS):
    """Eigenvalue of -D2 on the Fourier mode exp(i*theta*x): h^-2 (-w0 - 2 sum w_p cos p theta)."""
    w = fd_weights(radius)
    theta = np.asarray(theta, dtype=np.float64)
    s = -w[0] * np.ones_like(theta)
    for p in range(1, radius + 1):
        s = s - 2.0 * w[p] * np.cos(p * theta)
    return s / (h * h)


def _shift_zero(f, p, axis):
    """f shifted by p along axis (out[i] = f[i - p]) with zeros shifted in (Dirichlet)."""
    out = np.zeros_like(f)
    n = f.shape[axis]
    src = [slice(None)] * f.ndim
    dst = [slice(None)] * f.ndim
    if p >= 0:
        src[axis], dst[axis] = slice(0, n - p), slice(p, n)
    else:
        src[axis], dst[axis] = slice(-p, n), slice(0, n + p)
    out[tuple(dst)] = f[tuple(src)]
    return out


def second_diff_axis(f, h, axis, radius=RADIUS, bc="periodic"):
    """D2 along one axis, by summing shifted copies (np.roll when periodic, zero fill when
    Dirichlet)."""
    w = fd_weights(radius)
    out = w[0] * f
    for p in range(1, radius + 1):
        if bc == "periodic":
            out = out + w[p] * (np.roll(f, p, axis=axis) + np.roll(f, -p, axis=axis))
        else:
            out = out + w[p] * (_shift_zero(f, p, axis) + _shift_zero(f, -p, axis))
    return out / (h * h)


def laplacian(f, shape, h, radius=RADIUS, bc="periodic"):
    """Lap_h f for f of shape (N_d,) or (N_d, nvec); shape = (n0, n1, n2)."""
    n0, n1, n2 = shape
    f = np.asarray(f)
    vec = f.ndim == 1
    F = f.reshape(n2, n1, n0, -1)          # (z, y, x, nvec) since x is fastest
    out = (second_diff_axis(F, h, 2, radius, bc) + second_diff_axis(F, h, 1, radius, bc)
           + second_diff_axis(F, h, 0, radius, bc))
    out = out.reshape(n0 * n1 * n2, -1)
    return out[:, 0] if vec else out


def hamiltonian_apply(f, vloc, shape, h, radius=RADIUS, bc="periodic"):
    """H f = -1/2 Lap_h f + V_loc f (Eq. 4 for a local potential)."""
    f = np.asarray(f)
    v = vloc if f.ndim == 1 else vloc[:, None]
    return -0.5 * laplacian(f, shape, h, radius, bc) + v * f


def second_diff_dense_1d(n, h, radius=RADIUS, bc="periodic"):
    """Dense n x n matrix of D2: periodic (offsets that wrap onto the same point add up) or
    Dirichlet (offsets beyond the grid dropped)."""
    w = fd_weights(radius)
    D = np.zeros((n, n))
    for i in range(n):
        D[i, i] += w[0]
        for p in range(1, radius + 1):
            for j in (i + p, i - p):
                if bc == "periodic":
                    D[i, j % n] += w[p]
                elif 0 <= j < n:
                    D[i, j] += w[p]
    return D / (h * h)


def laplacian_dense(shape, h, radius=RADIUS, bc="periodic"):
    """Dense N_d x N_d Lap_h as a Kronecker sum (tiny grids only)."""
    n0, n1, n2 = shape
    Dx = second_diff_dense_1d(n0, h, radius, bc)
    Dy = second_diff_dense_1d(n1, h, radius, bc)
    Dz = second_diff_dense_1d(n2, h, radius, bc)
    Ix, Iy, Iz = np.eye(n0), np.eye(n1), np.eye(n2)
    # index i = x + n0*(y + n1*z): z is the slowest factor of the Kronecker product
    return (np.kron(Iz, np.kron(Iy, Dx)) + np.kron(Iz, np.kron(Dy, Ix))
            + np.kron(Dz, np.kron(Iy, Ix)))


def hamiltonian_dense(vloc, shape, h, radius=RADIUS, bc="periodic"):
    return -0.5 * laplacian_dense(shape, h, radius, bc) + np.diag(vloc)
