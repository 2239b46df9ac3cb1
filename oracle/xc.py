"""Local density approximation, spin-unpolarised (Sec. 2.2 lists LDA; the
workloads specify Slater exchange with the Perdew-Wang 1992 correlation).

Exchange (Slater/Dirac, textbook closed form):
    eps_x(rho) = -(3/4) (3 rho / pi)^(1/3),   v_x = (4/3) eps_x

Correlation (PW92 fit, unpolarised), with r_s = (3 / (4 pi rho))^(1/3):
    eps_c = -2A (1 + a1 r_s) ln(1 + 1 / (2A (b1 r_s^(1/2) + b2 r_s + b3 r_s^(3/2) + b4 r_s^2)))
    v_c   = eps_c - (r_s / 3) d eps_c / d r_s

The PW92 constants are not printed in the paper.  A is pinned by the exact
high-density coefficient (1 - ln 2) / pi^2 of the uniform electron gas, and
b2 = 2 A b1^2 by the absence of an r_s^(1/2) term from the exact high-density
expansion; the remaining fit constants (a1, b1, b3, b4) are parity unpinned
in this repository.
"""
from __future__ import annotations

import numpy as np

PW92_A = 0.031091
PW92_ALPHA1 = 0.21370
PW92_BETA = (7.5957, 3.5876, 1.6382, 0.49294)


def rs_of(rho):
    return (3.0 / (4.0 * np.pi * rho)) ** (1.0 / 3.0)


def slater_exchange(rho):
    """(eps_x, v_x) per electron / potential."""
    ex = -0.75 * (3.0 * rho / np.pi) ** (1.0 / 3.0)
    return ex, (4.0 / 3.0) * ex


def pw92_correlation(rs):
    """(eps_c, d eps_c / d r_s) at Wigner-Seitz radius r_s."""
    A, a1 = PW92_A, PW92_ALPHA1
    b1, b2, b3, b4 = PW92_BETA
    srs = np.sqrt(rs)
    Q0 = -2.0 * A * (1.0 + a1 * rs)
    Q1 = 2.0 * A * (b1 * srs + b2 * rs + b3 * rs * srs + b4 * rs * rs)
    dQ1 = A * (b1 / srs + 2.0 * b2 + 3.0 * b3 * srs + 4.0 * b4 * rs)
    lg = np.log(1.0 + 1.0 / Q1)
    ec = Q0 * lg
    dec = -2.0 * A * a1 * lg - Q0 * dQ1 / (Q1 * Q1 + Q1)
    return ec, dec


def lda(rho: np.ndarray, rho_floor: float = 1e-14):
    """(eps_xc, v_xc) of the unpolarised LDA at density max(rho, rho_floor)."""
    r = np.maximum(rho, rho_floor)
    ex, vx = slater_exchange(r)
    rs = rs_of(r)
    ec, dec = pw92_correlation(rs)
    vc = ec - rs / 3.0 * dec
    return ex + ec, vx + vc


# ---------------------------------------------------------------- spin (LSDA)
# Spin-resolved densities (eq. (1)-(2) carry a spin index).  Exchange obeys
# the exact spin-scaling relation E_x[rho_up, rho_dn] = (E_x[2 rho_up] +
# E_x[2 rho_dn]) / 2.  Correlation: the PW92 interpolation in the
# polarisation zeta = (rho_up - rho_dn) / rho,
#     eps_c(rs, zeta) = eps_c(rs, 0) + alpha_c(rs) f(zeta) / f''(0) (1 - zeta^4)
#                       + [eps_c(rs, 1) - eps_c(rs, 0)] f(zeta) zeta^4,
#     f(zeta) = ((1 + zeta)^(4/3) + (1 - zeta)^(4/3) - 2) / (2^(4/3) - 2),
# with eps_c(rs, 1) and -alpha_c(rs) of the same G(rs) form as eps_c(rs, 0).
# Their A constants are pinned by the exact high-density coefficients
# (1 - ln 2) / (2 pi^2) and 1 / (6 pi^2), and b2 = 2 A b1^2 in each fit by the
# absence of an r_s^(1/2) term; the other fit constants (a1, b1, b3, b4) are
# parity unpinned.

PW92_POL = (0.015545, 0.20548, (14.1189, 6.1977, 3.3662, 0.62517))      # eps_c(rs, 1)
PW92_MALPHA = (0.016887, 0.11125, (10.357, 3.6231, 0.88026, 0.49671))   # -alpha_c(rs)
FZ_DEN = 2.0 ** (4.0 / 3.0) - 2.0
FZ20 = 8.0 / (9.0 * FZ_DEN)                                             # f''(0)


def pw92_G(rs, A, a1, beta):
    """(G, dG/drs) of the PW92 form -2A (1 + a1 rs) ln(1 + 1 / (2A sum_j beta_j rs^(j/2)))."""
    b1, b2, b3, b4 = beta
    srs = np.sqrt(rs)
    Q0 = -2.0 * A * (1.0 + a1 * rs)
    Q1 = 2.0 * A * (b1 * srs + b2 * rs + b3 * rs * srs + b4 * rs * rs)
    dQ1 = A * (b1 / srs + 2.0 * b2 + 3.0 * b3 * srs + 4.0 * b4 * rs)
    lg = np.log(1.0 + 1.0 / Q1)
    return Q0 * lg, -2.0 * A * a1 * lg - Q0 * dQ1 / (Q1 * Q1 + Q1)


def spin_interp(zeta):
    """(f(zeta), f'(zeta))."""
    up, dn = 1.0 + zeta, 1.0 - zeta
    f = (up ** (4.0 / 3.0) + dn ** (4.0 / 3.0) - 2.0) / FZ_DEN
    df = (4.0 / 3.0) * (np.cbrt(up) - np.cbrt(dn)) / FZ_DEN
    return f, df


def lsda(rho_up: np.ndarray, rho_dn: np.ndarray, rho_floor: float = 1e-14):
    """(eps_xc, v_xc_up, v_xc_dn) of the spin-polarised LDA, each spin density
    floored at rho_floor / 2 (so that equal spins reduce to ``lda`` with its
    floor)."""
    ru = np.maximum(rho_up, 0.5 * rho_floor)
    rd = np.maximum(rho_dn, 0.5 * rho_floor)
    rho = ru + rd
    zeta = (ru - rd) / rho
    # exchange: per-spin Slater at twice the spin density
    exu, vxu = slater_exchange(2.0 * ru)
    exd, vxd = slater_exchange(2.0 * rd)
    ex = (ru * exu + rd * exd) / rho
    # correlation
    rs = rs_of(rho)
    e0, d0 = pw92_G(rs, PW92_A, PW92_ALPHA1, PW92_BETA)
    e1, d1 = pw92_G(rs, *PW92_POL)
    ma, dma = pw92_G(rs, *PW92_MALPHA)
    ac, dac = -ma, -dma
    f, df = spin_interp(zeta)
    z3, z4 = zeta ** 3, zeta ** 4
    ec = e0 + ac * f / FZ20 * (1.0 - z4) + (e1 - e0) * f * z4
    dec_rs = d0 + dac * f / FZ20 * (1.0 - z4) + (d1 - d0) * f * z4
    dec_z = ac / FZ20 * (df * (1.0 - z4) - 4.0 * z3 * f) + (e1 - e0) * (df * z4 + 4.0 * z3 * f)
    common = ec - rs / 3.0 * dec_rs
    vcu = common + (1.0 - zeta) * dec_z
    vcd = common - (1.0 + zeta) * dec_z
    return ex + ec, vxu + vcu, vxd + vcd
