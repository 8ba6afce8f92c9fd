"""Coulomb operator nu and nu^{1/2} on the periodic or Dirichlet grid (oracle).

Eq. 5 (Poisson): -1/(4 pi) Lap phi = rho, so on grid values nu = 4 pi (-Lap_h)^+,
the pseudo-inverse on the zero-mean subspace (the constant vector is the only
null vector of the periodic Lap_h).  Sec. 3 applies nu^{1/2} with the
Kronecker-product scheme: -D2_a = U_a diag(kappa_a) U_a^T per axis, so

    nu^{p/2} = (U_z (x) U_y (x) U_x) diag(s^p) (U_z (x) U_y (x) U_x)^T,
    s_{ijk} = sqrt(4 pi / (kappa_x,i + kappa_y,j + kappa_z,k)),  s = 0 on the
    mode with index 0 on every axis (the constant mode).

Here the 1D eigenbases come from a dense symmetric eigensolver of the periodic
1D matrix (eigenvalues ascending, so index 0 is the constant mode).  The dense
form (pseudo-inverse square root of the full N_d x N_d -Lap_h) is given for
tiny grids as an independent check.

Dirichlet grids (bc = "dirichlet"): -Lap_h is positive definite, nu = 4 pi (-Lap_h)^{-1} on the
whole space (the potential of a charge in a grounded box), every mode keeps its scale, and the
1D eigenbases are those of the Dirichlet 1D matrix (no closed form for the 12th-order stencil).
"""
import numpy as np

from . import fd


def eigbasis_1d(n, h, radius=fd.RADIUS, bc="periodic"):
    """(kappa, U): eigenvalues ascending and orthonormal eigenvectors of -D2 (n points)."""
    kappa, U = np.linalg.eigh(-fd.second_diff_dense_1d(n, h, radius, bc))
    return kappa, U


def coulomb_scale(shape, h, power=1, radius=fd.RADIUS, bc="periodic"):
    """s^power on the (z, y, x) mode grid; periodic: zero on the all-zero-index mode."""
    n0, n1, n2 = shape
    kx, _ = eigbasis_1d(n0, h, radius, bc)
    ky, _ = eigbasis_1d(n1, h, radius, bc)
    kz, _ = eigbasis_1d(n2, h, radius, bc)
    K = kz[:, None, None] + ky[None, :, None] + kx[None, None, :]
    if bc == "periodic":
        K[0, 0, 0] = 1.0                  # placeholder, overwritten below
    s = (4.0 * np.pi / K) ** (0.5 * power)
    if bc == "periodic":
        s[0, 0, 0] = 0.0
    return s


def nu_apply(V, shape, h, power=1, radius=fd.RADIUS, bc="periodic"):
    """nu^{power/2} V for V of shape (N_d,) or (N_d, nvec), via the three 1D transforms."""
    n0, n1, n2 = shape
    V = np.asarray(V, dtype=np.float64)
    vec = V.ndim == 1
    X = V.reshape(n2, n1, n0, -1)                 # (z, y, x, j)
    _, Ux = eigbasis_1d(n0, h, radius, bc)
    _, Uy = eigbasis_1d(n1, h, radius, bc)
    _, Uz = eigbasis_1d(n2, h, radius, bc)
    # forward transforms: coefficients along each axis, c_k = sum_x U[x, k] f_x
    X = np.einsum('zyxj,xa->zyaj', X, Ux)
    X = np.einsum('zyaj,yb->zbaj', X, Uy)
    X = np.einsum('zbaj,zc->cbaj', X, Uz)
    X = X * coulomb_scale(shape, h, power, radius, bc)[:, :, :, None]
    # inverse transforms
    X = np.einsum('cbaj,zc->zbaj', X, Uz)
    X = np.einsum('zbaj,yb->zyaj', X, Uy)
    X = np.einsum('zyaj,xa->zyxj', X, Ux)
    out = X.reshape(n0 * n1 * n2, -1)
    return out[:, 0] if vec else out


def nu_sqrt_dense(shape, h, radius=fd.RADIUS, bc="periodic"):
    """Dense nu^{1/2} = sqrt(4 pi) ((-Lap_h)^+)^{1/2} from the full eigendecomposition (tiny grids)."""
    lam, Q = np.linalg.eigh(-fd.laplacian_dense(shape, h, radius, bc))
    inv_sqrt = np.zeros_like(lam)
    if bc == "periodic":
        # exactly one null vector (the constant): drop the smallest eigenvalue only
        inv_sqrt[1:] = 1.0 / np.sqrt(lam[1:])
    else:
        inv_sqrt[:] = 1.0 / np.sqrt(lam)
    return np.sqrt(4.0 * np.pi) * (Q * inv_sqrt) @ Q.T
