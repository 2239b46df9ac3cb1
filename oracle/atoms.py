"""Atom-centred quantities on the periodic grid: pseudocharges, self and
overlap energies, atomic-density guess and nonlocal projectors.

Sec. 2.1 describes a local real-space electrostatics in which the ionic part
of the potential enters through the solution of a Poisson problem; the
pseudopotentials here are model ones whose local part V_I(r) = -Z erf(r/rc)/r
is exactly the potential of a normalised Gaussian charge, so the pseudocharge
is that Gaussian:

    b(x) = - sum_I sum_images Z_I (pi rc_I^2)^(-3/2) exp(-|x - R_I - nL|^2 / rc_I^2)

truncated at 8 rc_I.  The nonlocal part (Sec. 2.1: applied through its outer
product structure) is a sum of Kleinman-Bylander terms gamma chi chi^T with
continuum-normalised Gaussian radial parts (s and p).

Periodic images are handled by enumerating *unwrapped* integer grid indices
along each axis: index i stands for grid point (i mod N) in image cell
floor(i/N), and its displacement from the atom is i*h - R.  Every
(grid point, image) pair within the cutoff therefore appears exactly once.
"""
from __future__ import annotations

from dataclasses import dataclass
from math import erfc, pi, sqrt

import numpy as np
from scipy.special import erf as _erf


def ball_points(n, h, center, rmax):
    """All (flat grid index, displacement) pairs within distance ``rmax`` of
    ``center`` over all periodic images.

    Returns (flat, dx, dy, dz, r2) as 1D arrays."""
    ranges = []
    for d in range(3):
        lo = int(np.ceil((center[d] - rmax) / h[d]))
        hi = int(np.floor((center[d] + rmax) / h[d]))
        i = np.arange(lo, hi + 1)
        ranges.append((i, i * h[d] - center[d]))
    (ix, dx), (iy, dy), (iz, dz) = ranges
    DZ, DY, DX = np.meshgrid(dz, dy, dx, indexing="ij")
    IZ, IY, IX = np.meshgrid(iz, iy, ix, indexing="ij")
    r2 = DX * DX + DY * DY + DZ * DZ
    m = r2 <= rmax * rmax
    flat = np.mod(IX[m], n[0]) + n[0] * (np.mod(IY[m], n[1]) + n[1] * np.mod(IZ[m], n[2]))
    return flat.astype(np.int64), DX[m], DY[m], DZ[m], r2[m]


def pseudocharge(sys) -> np.ndarray:
    """b on the grid, flat (N_d,)."""
    nd = sys.nd
    b = np.zeros(nd)
    for I in range(sys.n_atoms):
        rc = sys.rc_loc[I]
        flat, _, _, _, r2 = ball_points(sys.n, sys.h, sys.pos[I], 8.0 * rc)
        vals = -sys.Z[I] * (pi * rc * rc) ** -1.5 * np.exp(-r2 / (rc * rc))
        b += np.bincount(flat, weights=vals, minlength=nd)
    return b


def local_potential_radial(Z, rc, r):
    """V(r) = -Z erf(r/rc)/r with its finite limit -2Z/(sqrt(pi) rc) at r = 0."""
    r = np.asarray(r, dtype=np.float64)
    out = np.empty_like(r)
    small = r < 1e-12
    out[small] = -2.0 * Z / (sqrt(pi) * rc)
    rr = r[~small]
    out[~small] = -Z * _erf(rr / rc) / rr
    return out


def self_energy(sys) -> float:
    """E_self = 1/2 sum_I  dV sum_x b_I(x) V_I(x), the trapezoidal-rule
    (Sec. 2.1) quadrature of the self-interaction of each isolated Gaussian
    pseudocharge, with the displacement taken from the atom's own (unwrapped)
    position."""
    e = 0.0
    for I in range(sys.n_atoms):
        rc = sys.rc_loc[I]
        _, _, _, _, r2 = ball_points(sys.n, sys.h, sys.pos[I], 8.0 * rc)
        bI = -sys.Z[I] * (pi * rc * rc) ** -1.5 * np.exp(-r2 / (rc * rc))
        VI = local_potential_radial(sys.Z[I], rc, np.sqrt(r2))
        e += 0.5 * sys.dV * float(np.sum(bI * VI))
    return e


def overlap_correction(sys, rmax: float = 10.0) -> float:
    """E_c = 1/2 sum_I sum_{J,n}' Z_I Z_J erfc(d / sqrt(rc_I^2 + rc_J^2)) / d:
    point-ion repulsion minus Gaussian-ion repulsion over all pairs and
    periodic images with d < rmax, excluding an atom with itself in the home
    cell."""
    L = np.asarray(sys.L)
    nimg = [int(np.ceil(rmax / L[d])) + 1 for d in range(3)]
    e = 0.0
    for I in range(sys.n_atoms):
        for J in range(sys.n_atoms):
            s = sqrt(sys.rc_loc[I] ** 2 + sys.rc_loc[J] ** 2)
            for a in range(-nimg[0], nimg[0] + 1):
                for b in range(-nimg[1], nimg[1] + 1):
                    for c in range(-nimg[2], nimg[2] + 1):
                        if I == J and a == 0 and b == 0 and c == 0:
                            continue
                        d = sys.pos[J] + np.array([a, b, c]) * L - sys.pos[I]
                        dist = float(np.sqrt(np.dot(d, d)))
                        if dist < rmax:
                            e += 0.5 * sys.Z[I] * sys.Z[J] * erfc(dist / s) / dist
    return e


def sad_density(sys) -> np.ndarray:
    """Superposition of atomic densities (Sec. 2.1, first SCF guess): one
    normalised Gaussian of width ``sad_width`` carrying Z_I electrons per atom
    (images summed, truncated at 8 widths), rescaled so that dV sum rho = N_e."""
    nd = sys.nd
    w = sys.sad_width
    rho = np.zeros(nd)
    for I in range(sys.n_atoms):
        flat, _, _, _, r2 = ball_points(sys.n, sys.h, sys.pos[I], 8.0 * w)
        vals = sys.Z[I] * (pi * w * w) ** -1.5 * np.exp(-r2 / (w * w))
        rho += np.bincount(flat, weights=vals, minlength=nd)
    rho *= sys.n_electrons / (sys.dV * rho.sum())
    return rho


@dataclass
class Projector:
    """Nonlocal projectors of one atom on its support.

    ``idx``: sorted unique flat grid indices; ``chi``: (4, len(idx)) values of
    chi_s, chi_px, chi_py, chi_pz (images summed); ``gamma``: (4,) energies
    (gamma_s, gamma_p, gamma_p, gamma_p)."""

    idx: np.ndarray
    chi: np.ndarray
    gamma: np.ndarray


def projectors(sys) -> list:
    """chi_s = N0 exp(-r^2/rc^2), chi_p{x,y,z} = N1 {x,y,z} exp(-r^2/rc^2) with
    N0 = (2/(pi rc^2))^(3/4), N1 = (2/rc) N0 (unit continuum norm), cut at
    r <= rcut_nl and summed over periodic images."""
    if sys.nl_lmax < 0:
        return []
    rc = sys.rc_nl
    N0 = (2.0 / (pi * rc * rc)) ** 0.75
    N1 = (2.0 / rc) * N0
    out = []
    for I in range(sys.n_atoms):
        flat, dx, dy, dz, r2 = ball_points(sys.n, sys.h, sys.pos[I], sys.rcut_nl)
        e = np.exp(-r2 / (rc * rc))
        vals = np.stack([N0 * e, N1 * dx * e, N1 * dy * e, N1 * dz * e])
        idx, inv = np.unique(flat, return_inverse=True)
        chi = np.zeros((4, idx.size))
        for k in range(4):
            chi[k] = np.bincount(inv, weights=vals[k], minlength=idx.size)
        g = sys.gamma[I]
        gamma = np.array([g[0], g[1], g[1], g[1]], dtype=np.float64)
        out.append(Projector(idx=idx, chi=chi, gamma=gamma))
    return out
