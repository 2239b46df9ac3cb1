"""Bloch-periodic k-points: complex orbitals of the form
psi(x + n L) = exp(i k . nL) psi(x) (test infrastructure: the CPU reference
the GPU k-point path is checked against).

Sec. 2.1: orbitals obey Bloch-periodic boundary conditions along extended
directions, and Brillouin-zone integration uses a set of k-points.  For one
k-point the Hamiltonian acting on a home-cell orbital is

    H_k psi = -1/2 Lap_h^k psi + V_eff psi + sum_I sum_lm gamma_Il chi~_Ilm <chi~_Ilm, psi>

where Lap_h^k is the same finite-difference stencil with the Bloch phase on
every neighbour that leaves the home cell (exp(+i k_d L_d) past the upper
face, exp(-i k_d L_d) past the lower face), and the projector of atom I is

    chi~_Ilm(x) = sum_s chi_lm(x + sL - R_I) exp(-i k . sL)

over the periodic images s (integer vectors) within the cutoff, with
<a, b> = dV sum conj(a) b.  Occupations: one Fermi level over all k with
weights w_k (sum w_k = 1), g_nk = 2 f_nk; the density is
rho = sum_k w_k sum_n g_nk |psi_nk|^2.  Blocks are complex arrays of shape
(ncol, N_d), one orbital per row.  Everything here is native complex
arithmetic (numpy complex128).
"""
from __future__ import annotations

from math import pi

import numpy as np

from . import chefsi, scf
from .fd import fd_weights


def bloch_laplacian(sys, Z: np.ndarray, k) -> np.ndarray:
    """Lap_h^k applied to each row of Z (complex, (ncol, N_d))."""
    nx, ny, nz = sys.n
    w = fd_weights(sys.fd_half_order)
    ncol = Z.shape[0]
    G = Z.reshape(ncol, nz, ny, nx)
    out = np.zeros_like(G)
    for axis_grid, d in ((3, 0), (2, 1), (1, 2)):
        n = sys.n[d]
        h2 = sys.h[d] ** 2
        idx = np.arange(n)
        acc = w[0] * G
        for q in range(1, len(w)):
            # neighbour i + q: past the upper face it is the image one cell up
            up = np.take(G, (idx + q) % n, axis=axis_grid)
            ph_up = np.where(idx + q >= n, np.exp(1j * k[d] * sys.L[d]), 1.0)
            dn = np.take(G, (idx - q) % n, axis=axis_grid)
            ph_dn = np.where(idx - q < 0, np.exp(-1j * k[d] * sys.L[d]), 1.0)
            shape = [1, 1, 1, 1]
            shape[axis_grid] = n
            acc = acc + w[q] * (up * ph_up.reshape(shape) + dn * ph_dn.reshape(shape))
        out = out + acc / h2
    return out.reshape(ncol, -1)


def projectors_k(sys, k):
    """Complex projectors of each atom: list of (idx, chi (4, npts) complex,
    gamma (4,)), with chi~ summed over images with phase exp(-i k . sL)."""
    if sys.nl_lmax < 0:
        return []
    rc = sys.rc_nl
    N0 = (2.0 / (pi * rc * rc)) ** 0.75
    N1 = (2.0 / rc) * N0
    nvec, h, L = np.asarray(sys.n), np.asarray(sys.h), np.asarray(sys.L)
    out = []
    for I in range(sys.n_atoms):
        R = sys.pos[I]
        axes = []
        for d in range(3):
            lo = int(np.ceil((R[d] - sys.rcut_nl) / h[d]))
            hi = int(np.floor((R[d] + sys.rcut_nl) / h[d]))
            axes.append(np.arange(lo, hi + 1))
        IZ, IY, IX = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
        ii = np.stack([IX.ravel(), IY.ravel(), IZ.ravel()])        # unwrapped indices
        dvec = ii * h[:, None] - R[:, None]
        r2 = np.sum(dvec * dvec, axis=0)
        m = r2 <= sys.rcut_nl ** 2
        ii, dvec, r2 = ii[:, m], dvec[:, m], r2[m]
        s = np.floor_divide(ii, nvec[:, None])                      # image of each point
        wrapped = ii - s * nvec[:, None]
        flat = wrapped[0] + nvec[0] * (wrapped[1] + nvec[1] * wrapped[2])
        phase = np.exp(-1j * np.sum(np.asarray(k)[:, None] * s * L[:, None], axis=0))
        e = np.exp(-r2 / (rc * rc))
        vals = np.stack([N0 * e, N1 * dvec[0] * e, N1 * dvec[1] * e, N1 * dvec[2] * e]) * phase[None, :]
        idx, inv = np.unique(flat, return_inverse=True)
        chi = np.zeros((4, idx.size), dtype=np.complex128)
        for q in range(4):
            np.add.at(chi[q], inv, vals[q])
        g = sys.gamma[I]
        out.append((idx, chi, np.array([g[0], g[1], g[1], g[1]], dtype=np.float64)))
    return out


def apply_H_k(sys, veff: np.ndarray, projs_k: list, Z: np.ndarray, k) -> np.ndarray:
    Z = np.atleast_2d(np.asarray(Z, dtype=np.complex128))
    Y = -0.5 * bloch_laplacian(sys, Z, k) + veff[None, :] * Z
    for idx, chi, gam in projs_k:
        C = sys.dV * (np.conj(chi) @ Z[:, idx].T)       # (4, ncol): <chi~, z>
        Y[:, idx] += (chi.T @ (gam[:, None] * C)).T
    return Y


def dense_H_k(sys, veff, projs_k, k) -> np.ndarray:
    """Dense H_k (N_d x N_d complex) column by column, for tiny grids."""
    E = np.eye(sys.nd, dtype=np.complex128)
    return apply_H_k(sys, veff, projs_k, E, k).T


def spectrum_bounds_k(sys, veff, projs_k):
    """The Gamma-point bounds hold for every k: the Bloch stencil's symbol is
    the same function at shifted wave numbers, and dV ||chi~||^2 bounds each
    rank-one nonlocal term."""
    from .fd import symbol
    spi = abs(float(symbol(np.pi, sys.fd_half_order)))
    kin = 0.5 * sum(spi / (hd * hd) for hd in sys.h)
    hi = kin + float(veff.max())
    lo = float(veff.min())
    for idx, chi, gam in projs_k:
        nrm = sys.dV * np.sum(np.abs(chi) ** 2, axis=1)
        hi += float(np.sum(np.maximum(gam, 0.0) * nrm))
        lo += float(np.sum(np.minimum(gam, 0.0) * nrm))
    return lo, hi


def chebyshev_filter_k(sys, veff, projs_k, Z, k, m: int, a: float, b: float, a0: float) -> np.ndarray:
    """The scaled Chebyshev filter of ``chefsi.chebyshev_filter`` with H_k."""
    e = (b - a) / 2.0
    c = (b + a) / 2.0
    sigma = e / (a0 - c)
    tau = 2.0 / sigma
    Yprev = Z
    Y = (sigma / e) * (apply_H_k(sys, veff, projs_k, Z, k) - c * Z)
    for _ in range(2, m + 1):
        sigma_new = 1.0 / (tau - sigma)
        Ynew = (2.0 * sigma_new / e) * (apply_H_k(sys, veff, projs_k, Y, k) - c * Y) - (sigma * sigma_new) * Yprev
        Yprev, Y, sigma = Y, Ynew, sigma_new
    return Y


def rayleigh_ritz_k(sys, veff, projs_k, Y, k):
    """Complex Cholesky-QR (M_ij = dV <y_i, y_j>, M = L L^H, rows
    X = conj(L)^-1 Y so that dV <x_i, x_j> = delta_ij) and Rayleigh-Ritz with
    the Hermitian projected H_k; returns (X, lam)."""
    M = sys.dV * (np.conj(Y) @ Y.T)
    Lc = np.linalg.cholesky(M)
    piv = np.real(np.diag(Lc)) ** 2
    if np.any(~np.isfinite(piv)) or np.any(piv <= chefsi.PIVOT_RTOL * np.real(np.diag(M))):
        raise chefsi.NotSPD("numerically rank-deficient block")
    X = np.linalg.solve(np.conj(Lc), Y)
    HX = apply_H_k(sys, veff, projs_k, X, k)
    Hs = sys.dV * (np.conj(X) @ HX.T)
    Hs = 0.5 * (Hs + np.conj(Hs.T))
    lam, Q = np.linalg.eigh(Hs)
    return Q.T @ X, lam


def occupations_k(lams, wk, n_electrons: float, kT: float, tol: float = 1e-13, max_iter: int = 500):
    """One Fermi level over all k: sum_k w_k sum_n 2 f(lam_nk) = N_e.
    Returns (mu, [g_k])."""
    allv = np.concatenate([np.asarray(l, dtype=np.float64) for l in lams])
    lo = float(allv.min()) - 40.0 * kT
    hi = float(allv.max()) + 40.0 * kT
    mu = 0.5 * (lo + hi)
    for _ in range(max_iter):
        mu = 0.5 * (lo + hi)
        n = sum(w * 2.0 * float(np.sum(scf.fermi(l, mu, kT))) for l, w in zip(lams, wk))
        if abs(n - n_electrons) < tol:
            break
        if n < n_electrons:
            lo = mu
        else:
            hi = mu
        if not (lo < 0.5 * (lo + hi) < hi):
            break
    return mu, [2.0 * scf.fermi(l, mu, kT) for l in lams]


def density_k(Xs, gs, wk) -> np.ndarray:
    return sum(w * np.sum(g[:, None] * np.abs(X) ** 2, axis=0) for X, g, w in zip(Xs, gs, wk))


def scf_k(sys, kpts, wk, Z0s, rho0=None, max_iter: int = 50, tol: float = 1e-10, st=None, n_first: int = None,
          degree: int = None, beta: float = None):
    """The SCF schedule of ``scf.scf`` with one CheFSI block per k-point
    (filter bounds tracked per k), occupations with one Fermi level over all
    k, and the k-weighted density; linear mixing with the Kerker-type
    preconditioner when sys.kerker_q0 > 0, or periodic Pulay mixing when
    sys.pulay_history > 0 (as in ``scf.scf``).  Parity unpinned away from the
    fixed point, as for ``scf.scf``."""
    st = st or scf.setup(sys)
    n_first = sys.n_first if n_first is None else n_first
    m = sys.cheb_degree if degree is None else degree
    beta = sys.mix_beta if beta is None else beta
    from . import atoms
    rho_in = atoms.sad_density(sys) if rho0 is None else rho0.copy()
    Xs = [np.array(Z, dtype=np.complex128) for Z in Z0s]
    pk = [projectors_k(sys, k) for k in kpts]
    ab = [None] * len(kpts)
    pulay = None
    if getattr(sys, "pulay_history", 0) > 0:
        pulay = scf.PeriodicPulay(sys.pulay_history, sys.pulay_period, beta, sys, getattr(sys, "kerker_q0", 0.0),
                                  bool(getattr(sys, "pulay_restart", 0)))
    hist = []
    for it in range(max_iter):
        phi, exc, vxc, veff = scf.potential(sys, st, rho_in)
        lams = []
        for q, k in enumerate(kpts):
            lo, hi = spectrum_bounds_k(sys, veff, pk[q])
            if it == 0:
                Xs[q], lam = rayleigh_ritz_k(sys, veff, pk[q], Xs[q], k)
                a, a0 = float(lam[-1]), lo
            else:
                a, a0 = ab[q]
            for _ in range(n_first if it == 0 else 1):
                Y = chebyshev_filter_k(sys, veff, pk[q], Xs[q], k, m, a, hi, a0)
                Xs[q], lam = rayleigh_ritz_k(sys, veff, pk[q], Y, k)
                a, a0 = float(lam[-1]), float(lam[0])
            ab[q] = (a, a0)
            lams.append(lam)
        mu, gs = occupations_k(lams, wk, sys.n_electrons, sys.kT)
        rho_out = density_k(Xs, gs, wk)
        # band and entropy terms with the k weights
        band = float(sum(w * np.sum(g * l) for g, l, w in zip(gs, lams, wk)))
        ent = float(sum(w * scf.entropy_term(g, sys.kT) for g, w in zip(gs, wk)))
        dV = sys.dV
        terms = {
            "band": band,
            "exc": dV * float(np.sum(rho_in * exc)),
            "vxc_dc": -dV * float(np.sum(rho_in * vxc)),
            "elec": 0.5 * dV * float(np.sum((st.b - rho_in) * phi)),
            "self": -st.e_self,
            "corr": st.e_c,
            "entropy": ent,
        }
        terms["free"] = sum(terms.values())
        res = float(np.linalg.norm(rho_out - rho_in) / np.linalg.norm(rho_out))
        hist.append(dict(it=it, residual=res, mu=mu, lam=[l.copy() for l in lams], **terms))
        rho_prev = rho_in
        if pulay is not None:
            rho_in = pulay.step(rho_in, rho_out - rho_in)
        else:
            rho_in = scf.mix(rho_in, rho_out, beta, sys, getattr(sys, "kerker_q0", 0.0))
        if res < tol:
            break
    return dict(X=Xs, lam=lams, g=gs, mu=mu, rho_in=rho_prev, rho_out=rho_out, history=hist)
