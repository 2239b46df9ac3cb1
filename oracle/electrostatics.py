"""Electrostatic potential from the periodic Poisson problem (Sec. 2.1: the sum
of ionic and Hartree potentials solves a Poisson problem, discretised with the
same finite-difference Laplacian; periodic boundary conditions in extended
directions).

    -Delta_h phi = 4 pi (rho + b - mean(rho + b)),   mean(phi) = 0

The discrete periodic Laplacian is diagonal in the discrete Fourier basis, with
eigenvalue S(k) = sum_d h_d^-2 s(2 pi j_d / N_d) where s is the 1D stencil
symbol.  The oracle solves the discrete problem exactly in that basis (FFT as
a library step): phi_hat = -4 pi r_hat / S, phi_hat(0) = 0.  This is an
independent route to the same discrete solution an iterative stencil solver
reaches (the paper uses AAR; any convergent solver of the same linear system
gives the same phi).
"""
from __future__ import annotations

import numpy as np

from .fd import symbol


def fd_symbol_3d(sys) -> np.ndarray:
    """S on the FFT grid, shape (Nz, Ny, Nx)."""
    nx, ny, nz = sys.n
    hx, hy, hz = sys.h
    sx = symbol(2 * np.pi * np.arange(nx) / nx, sys.fd_half_order) / (hx * hx)
    sy = symbol(2 * np.pi * np.arange(ny) / ny, sys.fd_half_order) / (hy * hy)
    sz = symbol(2 * np.pi * np.arange(nz) / nz, sys.fd_half_order) / (hz * hz)
    return sz[:, None, None] + sy[None, :, None] + sx[None, None, :]


def solve_poisson(sys, charge: np.ndarray) -> np.ndarray:
    """phi (flat) solving -Delta_h phi = 4 pi (charge - mean(charge)), mean 0."""
    nx, ny, nz = sys.n
    r = charge.reshape(nz, ny, nx)
    r = r - r.mean()
    rh = np.fft.fftn(r)
    S = fd_symbol_3d(sys)
    S[0, 0, 0] = 1.0
    ph = -4.0 * np.pi * rh / S
    ph[0, 0, 0] = 0.0
    return np.real(np.fft.ifftn(ph)).reshape(-1)


def hartree_ionic_potential(sys, rho: np.ndarray, b: np.ndarray) -> np.ndarray:
    """phi for electron density rho and pseudocharge b."""
    return solve_poisson(sys, rho + b)
