"""Frequency quadrature for the imaginary-frequency integral (oracle).

Sec. 3: the integral over omega in Eq. 1 / Eq. 10 is approximated by
Gauss-Legendre quadrature, and the loop over frequencies runs from the highest
frequency to the lowest (Algorithm 1).  The paper does not state how [-1, 1]
is mapped onto [0, inf); the rational map used here is

    omega = omega0 (1 + t) / (1 - t),   d omega = 2 omega0 / (1 - t)^2 dt,

so a node t_m with Legendre weight w_m gives omega_m and weight
W_m = w_m 2 omega0 / (1 - t_m)^2.
"""
import numpy as np


def frequency_grid(n=8, omega0=1.0):
    """(omega, weight), both length n, ordered from the highest frequency to the lowest."""
    t, w = np.polynomial.legendre.leggauss(n)
    omega = omega0 * (1.0 + t) / (1.0 - t)
    weight = w * 2.0 * omega0 / (1.0 - t) ** 2
    order = np.argsort(-omega)
    return omega[order], weight[order]
