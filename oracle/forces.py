"""Hellmann-Feynman atomic forces (test infrastructure: the CPU reference the
GPU forces are checked against).

The paper computes atomic forces from the self-consistent ground state
(Sec. 2: structural relaxation and molecular dynamics use the
Hellmann-Feynman forces).  Here they are the exact negative gradient, with
respect to the atom positions, of the discrete free energy of ``scf``
evaluated at self-consistency, where the orbitals, occupations and density
are stationary and only the explicit position dependence contributes:

  electrostatics  E_el = 1/2 dV sum (rho + b) phi  with  -Lap_h phi = 4 pi (rho + b):
      F_I += dV sum_x phi(x) grad b_I(x - R_I)
  self energy     -E_self = -1/2 dV sum over the atom's ball of b_I V_I:
      F_I -= 1/2 dV sum grad(b_I V_I)(x - R_I)
  overlap         E_c = 1/2 sum_I sum_{J,n}' Z_I Z_J u(d),  u(d) = erfc(d / s) / d:
      F_I += sum_{J,n}' Z_I Z_J u'(d) (R_J + nL - R_I) / d
  nonlocal        E_nl = sum_n w_n sum_{I,k} gamma_Ik (dV chi_Ik^T psi_n)^2:
      F_I += 2 sum_n w_n sum_k gamma_Ik (dV chi_Ik^T psi_n)(dV (grad chi_Ik)^T psi_n)

with grad b = b (-2 d / rc^2), grad V = V'(r) d / r, grad chi_s = chi_s
(-2 d / rc^2), grad (N1 d_a e) = N1 e (e_a - 2 d_a d / rc^2), every sum
over the same (grid point, image) pairs the energy uses.  The weights w_n
are the occupations g_n = 2 f_n (spin-unpolarised) or f_n^s per spin block.
The truncation spheres (8 rc for b, rcut_nl for chi) are fixed in
displacement, so points crossing them are not differentiated: the pins use
cutoffs at which the truncated tails are below rounding.
"""
from __future__ import annotations

from math import erfc, pi, sqrt

import numpy as np
from scipy.special import erf as _erf

from . import atoms


def _atoms(sys, atoms_subset):
    return range(sys.n_atoms) if atoms_subset is None else atoms_subset


def local_forces(sys, phi: np.ndarray, atoms_subset=None) -> np.ndarray:
    """Electrostatic (pseudocharge) plus self-energy part, (n_atoms, 3); rows
    outside ``atoms_subset`` (all atoms when None) are left zero."""
    F = np.zeros((sys.n_atoms, 3))
    for I in _atoms(sys, atoms_subset):
        Z, rc = sys.Z[I], sys.rc_loc[I]
        flat, dx, dy, dz, r2 = atoms.ball_points(sys.n, sys.h, sys.pos[I], 8.0 * rc)
        b = -Z * (pi * rc * rc) ** -1.5 * np.exp(-r2 / (rc * rc))
        r = np.sqrt(r2)
        V = atoms.local_potential_radial(Z, rc, r)
        # V'(r) = Z erf(r/rc) / r^2 - Z (2 / (sqrt(pi) rc)) exp(-r^2/rc^2) / r, and V'(r)/r -> finite
        small = r < 1e-8
        dVr = np.empty_like(r)        # V'(r) / r
        rr = r[~small]
        dVr[~small] = (Z * _erf(rr / rc) / rr ** 2 - Z * 2.0 / (sqrt(pi) * rc) * np.exp(-rr * rr / (rc * rc)) / rr) / rr
        dVr[small] = 4.0 * Z / (3.0 * sqrt(pi) * rc ** 3)
        d = np.stack([dx, dy, dz])
        gb = b * (-2.0 / (rc * rc)) * d
        gV = dVr * d
        F[I] = sys.dV * (np.sum(phi[flat] * gb, axis=1) - 0.5 * np.sum(V * gb + b * gV, axis=1))
    return F


def overlap_forces(sys, rmax: float = 10.0, atoms_subset=None) -> np.ndarray:
    """-dE_c/dR_I over the pairs and images of ``atoms.overlap_correction``."""
    L = np.asarray(sys.L)
    nimg = [int(np.ceil(rmax / L[d])) + 1 for d in range(3)]
    F = np.zeros((sys.n_atoms, 3))
    for I in _atoms(sys, atoms_subset):
        for J in range(sys.n_atoms):
            s = sqrt(sys.rc_loc[I] ** 2 + sys.rc_loc[J] ** 2)
            for a in range(-nimg[0], nimg[0] + 1):
                for b in range(-nimg[1], nimg[1] + 1):
                    for c in range(-nimg[2], nimg[2] + 1):
                        if I == J and a == 0 and b == 0 and c == 0:
                            continue
                        v = sys.pos[J] + np.array([a, b, c]) * L - sys.pos[I]
                        dist = float(np.sqrt(np.dot(v, v)))
                        if dist < rmax:
                            du = -erfc(dist / s) / dist ** 2 - 2.0 / (sqrt(pi) * s) * np.exp(-(dist / s) ** 2) / dist
                            F[I] += sys.Z[I] * sys.Z[J] * du * v / dist
    return F


def nonlocal_forces(sys, blocks, weights, atoms_subset=None) -> np.ndarray:
    """blocks: orbital blocks (rows are orbitals); weights: their occupation
    weights (g_n, or f_n^s per spin block)."""
    F = np.zeros((sys.n_atoms, 3))
    if sys.nl_lmax < 0:
        return F
    rc = sys.rc_nl
    N0 = (2.0 / (pi * rc * rc)) ** 0.75
    N1 = (2.0 / rc) * N0
    for I in _atoms(sys, atoms_subset):
        flat, dx, dy, dz, r2 = atoms.ball_points(sys.n, sys.h, sys.pos[I], sys.rcut_nl)
        e = np.exp(-r2 / (rc * rc))
        d = np.stack([dx, dy, dz])
        chi = [N0 * e, N1 * dx * e, N1 * dy * e, N1 * dz * e]
        grad = [N0 * e * (-2.0 / (rc * rc)) * d]
        for a in range(3):
            ga = N1 * e * (-2.0 * d[a] / (rc * rc)) * d
            ga[a] += N1 * e
            grad.append(ga)
        g = sys.gamma[I]
        gam = [g[0], g[1], g[1], g[1]]
        for X, w in zip(blocks, weights):
            Xs = X[:, flat]                                     # (n, points)
            for k in range(4):
                P = sys.dV * (Xs @ chi[k])                      # (n,)
                D = sys.dV * (Xs @ grad[k].T)                   # (n, 3)
                F[I] += 2.0 * gam[k] * np.sum((w * P)[:, None] * D, axis=0)
    return F


def forces(sys, phi: np.ndarray, blocks, weights, atoms_subset=None) -> np.ndarray:
    """Total Hellmann-Feynman force (n_atoms, 3) at the density whose
    electrostatic potential is phi and the orbital blocks with weights (rows
    of ``atoms_subset`` only, when given)."""
    return (local_forces(sys, phi, atoms_subset) + overlap_forces(sys, atoms_subset=atoms_subset)
            + nonlocal_forces(sys, blocks, weights, atoms_subset))
