"""High-order centred finite differences on a periodic grid.

Sec. 2.1: the equations are discretised on a uniform real-space grid with a
high-order centred finite-difference approximation of the Laplacian.  The
order is not stated in the paper; the workloads use 12th order (half-width
n_o = 6).  The weights below are the standard centred second-derivative
weights of order 2*n_o:

    w_q = 2 (-1)^(q+1) (n_o!)^2 / (q^2 (n_o-q)! (n_o+q)!),   q = 1..n_o
    w_0 = -2 sum_q w_q

so that  f''(x) ~ h^-2 [w_0 f(x) + sum_q w_q (f(x+qh) + f(x-qh))].
"""
from __future__ import annotations

from fractions import Fraction
from math import factorial

import numpy as np


def fd_weights_exact(n_o: int) -> list:
    """Exact rational weights [w_0, w_1, ..., w_{n_o}]."""
    w = [Fraction(0)] * (n_o + 1)
    for q in range(1, n_o + 1):
        num = 2 * (-1) ** (q + 1) * factorial(n_o) ** 2
        den = q * q * factorial(n_o - q) * factorial(n_o + q)
        w[q] = Fraction(num, den)
    w[0] = -2 * sum(w[1:])
    return w


def fd_weights(n_o: int) -> np.ndarray:
    return np.array([float(v) for v in fd_weights_exact(n_o)], dtype=np.float64)


def symbol(theta, n_o: int):
    """Fourier symbol s(theta) = w_0 + 2 sum_q w_q cos(q theta) of the 1D
    stencil: applied to exp(i j theta) it returns s(theta) exp(i j theta)."""
    w = fd_weights(n_o)
    theta = np.asarray(theta, dtype=np.float64)
    out = np.full(theta.shape, w[0])
    for q in range(1, n_o + 1):
        out = out + 2.0 * w[q] * np.cos(q * theta)
    return out


def laplacian(f: np.ndarray, h, n_o: int) -> np.ndarray:
    """Periodic discrete Laplacian of grid functions.

    ``f`` has shape (..., Nz, Ny, Nx) (x fastest, matching the flat index
    ix + Nx*(iy + Ny*iz)); ``h = (hx, hy, hz)``."""
    w = fd_weights(n_o)
    out = np.zeros_like(f)
    # axis -1 is x, -2 is y, -3 is z
    for axis, hd in ((-1, h[0]), (-2, h[1]), (-3, h[2])):
        acc = w[0] * f
        for q in range(1, n_o + 1):
            acc = acc + w[q] * (np.roll(f, q, axis=axis) + np.roll(f, -q, axis=axis))
        out += acc / (hd * hd)
    return out
