"""Matrix-free Kohn-Sham Hamiltonian applied to a block of orbitals.

Sec. 2 eq. (1): H = -1/2 nabla^2 + V_eff (Gamma point, real orbitals).  Sec. 2.1:
H-times-vector products are matrix-free, using the finite-difference stencil
for the Laplacian and the outer-product form of the nonlocal pseudopotential:

    H x = -1/2 Delta_h x + V_eff . x + sum_I sum_lm gamma_Il chi_Ilm (dV chi_Ilm^T x)

with dV = hx*hy*hz the trapezoidal weight (Sec. 2.1).

Blocks are arrays of shape (ncol, N_d): row j is orbital j.
"""
from __future__ import annotations

import numpy as np

from .fd import fd_weights, laplacian, symbol


def apply_H(sys, veff: np.ndarray, projs: list, X: np.ndarray) -> np.ndarray:
    nx, ny, nz = sys.n
    X = np.atleast_2d(X)
    ncol = X.shape[0]
    Xg = X.reshape(ncol, nz, ny, nx)
    Y = (-0.5 * laplacian(Xg, sys.h, sys.fd_half_order)).reshape(ncol, -1)
    Y += veff[None, :] * X
    for P in projs:
        Xs = X[:, P.idx]                       # (ncol, npts)
        C = sys.dV * (P.chi @ Xs.T)            # (4, ncol)  projections
        D = P.gamma[:, None] * C               # scaled by the projector energies
        Y[:, P.idx] += (P.chi.T @ D).T
    return Y


def nonlocal_norms(sys, projs: list) -> list:
    """dV * ||chi_Ilm||^2 for each atom: the single non-zero eigenvalue of
    dV chi chi^T for that projector."""
    return [sys.dV * np.sum(P.chi * P.chi, axis=1) for P in projs]


def spectrum_bounds(sys, veff: np.ndarray, projs: list):
    """Deterministic bounds lo <= spec(H) <= hi.

    The Laplacian part is bounded by 0 <= -1/2 Delta_h <= 1/2 sum_d |s(pi)| / h_d^2
    (s the stencil symbol, which attains its most negative value at theta = pi
    for these weights), V_eff by its extrema, and each rank-one nonlocal term
    by min(gamma, 0) and max(gamma, 0) times dV ||chi||^2."""
    spi = abs(float(symbol(np.pi, sys.fd_half_order)))
    kin = 0.5 * sum(spi / (hd * hd) for hd in sys.h)
    nl_hi = 0.0
    nl_lo = 0.0
    for P, nrm in zip(projs, nonlocal_norms(sys, projs)):
        nl_hi += float(np.sum(np.maximum(P.gamma, 0.0) * nrm))
        nl_lo += float(np.sum(np.minimum(P.gamma, 0.0) * nrm))
    hi = kin + float(veff.max()) + nl_hi
    lo = float(veff.min()) + nl_lo
    return lo, hi


def dense_H(sys, veff: np.ndarray, projs: list) -> np.ndarray:
    """Dense N_d x N_d matrix of H built column by column from H e_j (only for
    tiny grids)."""
    nd = sys.nd
    I = np.eye(nd)
    H = np.empty((nd, nd))
    step = 256
    for j0 in range(0, nd, step):
        cols = I[j0:j0 + step]
        H[:, j0:j0 + step] = apply_H(sys, veff, projs, cols).T
    return H
