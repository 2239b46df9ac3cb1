"""Chebyshev-filtered subspace iteration steps (Sec. 2.1: in every SCF iteration
a partial diagonalisation by CheFSI, with several filtering passes in the first
iteration).  The filter and Rayleigh-Ritz procedure are the standard ones of
the CheFSI method the paper cites; they are written out here step by step.

Scaled Chebyshev filter of degree m on the interval [a, b] to be damped, with
a0 < a the point where the filter is normalised to one:

    e = (b - a)/2,  c = (b + a)/2,  sigma_1 = e / (a0 - c),  tau = 2 / sigma_1
    Y_1 = (sigma_1 / e) (H X - c X)
    for k = 2..m:
        sigma_k = 1 / (tau - sigma_{k-1})
        Y_k = (2 sigma_k / e) (H Y_{k-1} - c Y_{k-1}) - sigma_{k-1} sigma_k Y_{k-2}
    (Y_0 = X)

On an eigenvector with eigenvalue lam the result is
T_m((lam - c)/e) / T_m((a0 - c)/e) times the vector.

Orthonormalisation and Rayleigh-Ritz (dV-weighted inner product, Sec. 2.1
trapezoidal rule):

    M = dV Y^T Y = R^T R (Cholesky),  X = Y R^-1
    Hs = dV X^T (H X), symmetrised,  Hs = Q diag(lam) Q^T (ascending),  X <- X Q
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import solve_triangular

from .hamiltonian import apply_H


def chebyshev_filter(sys, veff, projs, X, m: int, a: float, b: float, a0: float) -> np.ndarray:
    e = (b - a) / 2.0
    c = (b + a) / 2.0
    sigma = e / (a0 - c)
    tau = 2.0 / sigma
    Yprev = X
    Y = (sigma / e) * (apply_H(sys, veff, projs, X) - c * X)
    for _ in range(2, m + 1):
        sigma_new = 1.0 / (tau - sigma)
        Ynew = (2.0 * sigma_new / e) * (apply_H(sys, veff, projs, Y) - c * Y) - (sigma * sigma_new) * Yprev
        Yprev = Y
        Y = Ynew
        sigma = sigma_new
    return Y


class NotSPD(RuntimeError):
    pass


# Cholesky pivots at or below this fraction of their diagonal entry are
# treated as zero (about 64 units of double-precision rounding).
PIVOT_RTOL = 64.0 * np.finfo(np.float64).eps


def orthonormalize(sys, Y: np.ndarray) -> np.ndarray:
    """X = Y R^-1 with dV Y^T Y = R^T R; rows of the returned block are
    dV-orthonormal."""
    M = sys.dV * (Y @ Y.T)                 # rows are orbitals: M_ij = dV <y_i, y_j>
    try:
        Lc = np.linalg.cholesky(M)         # M = Lc Lc^T, R = Lc^T
    except np.linalg.LinAlgError as exc:
        raise NotSPD(str(exc))
    # a pivot that is pure rounding noise (relative to its diagonal entry)
    # means the block is numerically rank deficient
    piv = np.diag(Lc) ** 2
    if np.any(~np.isfinite(piv)) or np.any(piv <= PIVOT_RTOL * np.diag(M)):
        raise NotSPD("numerically rank-deficient block")
    # X^T = Y^T R^-1  <=>  X = R^-T Y = Lc^-1 Y
    return solve_triangular(Lc, Y, lower=True)


def rayleigh_ritz(sys, veff, projs, Y: np.ndarray):
    """Returns (X, lam): Ritz vectors (rows, dV-orthonormal) and ascending Ritz
    values of the span of the rows of Y."""
    X = orthonormalize(sys, Y)
    HX = apply_H(sys, veff, projs, X)
    Hs = sys.dV * (X @ HX.T)
    Hs = 0.5 * (Hs + Hs.T)
    lam, Q = np.linalg.eigh(Hs)
    return Q.T @ X, lam
