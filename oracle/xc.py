"""Local density approximation, spin-unpolarised (Sec. 2.2 lists LDA; the
workloads specify Slater exchange with the Perdew-Wang 1992 correlation).

Exchange (Slater/Dirac, textbook closed form):
    eps_x(rho) = -(3/4) (3 rho / pi)^(1/3),   v_x = (4/3) eps_x

Correlation (PW92 fit, unpolarised), with r_s = (3 / (4 pi rho))^(1/3):
    eps_c = -2A (1 + a1 r_s) ln(1 + 1 / (2A (b1 r_s^(1/2) + b2 r_s + b3 r_s^(3/2) + b4 r_s^2)))
    v_c   = eps_c - (r_s / 3) d eps_c / d r_s

The PW92 constants are not printed in the paper.  A is pinned by the exact
high-density coefficient (1 - ln 2) / pi^2 of the uniform electron gas; the
remaining fit constants (a1, b1..b4) are parity unpinned in this repository.
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
