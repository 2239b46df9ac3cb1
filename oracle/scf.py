"""Occupations, density, energy, mixing and the SCF schedule.

Sec. 2 eq. (2): rho(x) = sum_n g_n |psi_n(x)|^2 with Fermi-Dirac occupations;
spin-unpolarised, so g_n = 2 f_n with f_n = 1 / (1 + exp((lam_n - mu) / kT))
and mu fixed by sum_n g_n = N_e.

Sec. 2.1: the ground state is the fixed point of the SCF iteration; the first
iteration starts from a superposition of atomic densities and performs several
CheFSI filtering passes, later iterations one.  The paper accelerates the
iteration with restarted periodic Pulay mixing and a real-space
preconditioner; the workloads here prescribe simple linear mixing
rho_in <- rho_in + beta (rho_out - rho_in), optionally with the residual
filtered by the Kerker-type preconditioner P = (-Lap_h)(-Lap_h + q0^2)^-1
(needed against charge sloshing in the larger cells; q0 = 0 is plain linear
mixing).

Energy: Harris-Foulkes free energy evaluated at the input density,
    F = sum_n g_n lam_n + dV sum rho_in eps_xc - dV sum rho_in v_xc
        + 1/2 dV sum (b - rho_in) phi - E_self + E_c
        + 2 kT sum_n [f_n ln f_n + (1 - f_n) ln(1 - f_n)]
(band energy minus double counting, electrostatics of rho_in + b with the
Gaussian self-energies removed and the point-ion overlap correction added,
and the -TS electronic entropy term of finite-temperature DFT).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import atoms, chefsi, electrostatics, hamiltonian, xc


def fermi(lam, mu, kT):
    """Overflow-safe Fermi-Dirac function."""
    x = (np.asarray(lam, dtype=np.float64) - mu) / kT
    out = np.empty_like(x)
    pos = x > 0
    ep = np.exp(-x[pos])
    out[pos] = ep / (1.0 + ep)
    out[~pos] = 1.0 / (1.0 + np.exp(x[~pos]))
    return out


class FermiError(RuntimeError):
    pass


def occupations(lam, n_electrons: float, kT: float, tol: float = 1e-13, max_iter: int = 500):
    """mu by bisection on [lam_min - 40 kT, lam_max + 40 kT] until
    |sum g - N_e| < tol (or the bracket stops shrinking); returns (mu, g)."""
    lam = np.asarray(lam, dtype=np.float64)
    if n_electrons > 2.0 * lam.size or n_electrons <= 0.0:
        raise FermiError("electron count outside (0, 2 N_s]")
    lo = float(lam.min()) - 40.0 * kT
    hi = float(lam.max()) + 40.0 * kT
    mu = 0.5 * (lo + hi)
    for _ in range(max_iter):
        mu = 0.5 * (lo + hi)
        n = 2.0 * float(np.sum(fermi(lam, mu, kT)))
        if abs(n - n_electrons) < tol:
            break
        if n < n_electrons:
            lo = mu
        else:
            hi = mu
        if not (lo < 0.5 * (lo + hi) < hi):
            break
    return mu, 2.0 * fermi(lam, mu, kT)


def density(X: np.ndarray, g: np.ndarray) -> np.ndarray:
    """rho = sum_n g_n X_n^2 (rows of X are orbitals)."""
    return np.sum(g[:, None] * X * X, axis=0)


def entropy_term(g, kT):
    """2 kT sum [f ln f + (1-f) ln(1-f)] with f = g/2 (0 ln 0 = 0)."""
    f = np.asarray(g) / 2.0
    s = 0.0
    for v in f:
        if 0.0 < v < 1.0:
            s += v * np.log(v) + (1.0 - v) * np.log(1.0 - v)
    return 2.0 * kT * s


@dataclass
class Setup:
    """Geometry-derived quantities of one system."""
    b: np.ndarray
    projs: list
    e_self: float
    e_c: float


def setup(sys) -> Setup:
    return Setup(
        b=atoms.pseudocharge(sys),
        projs=atoms.projectors(sys),
        e_self=atoms.self_energy(sys),
        e_c=atoms.overlap_correction(sys),
    )


def potential(sys, st: Setup, rho: np.ndarray):
    """(phi, eps_xc, v_xc, V_eff) for input density rho."""
    phi = electrostatics.hartree_ionic_potential(sys, rho, st.b)
    exc, vxc = xc.lda(rho, sys.rho_floor)
    return phi, exc, vxc, phi + vxc


def energy_terms(sys, st: Setup, rho_in, phi, exc, vxc, lam, g):
    dV = sys.dV
    t = {
        "band": float(np.sum(g * lam)),
        "exc": dV * float(np.sum(rho_in * exc)),
        "vxc_dc": -dV * float(np.sum(rho_in * vxc)),
        "elec": 0.5 * dV * float(np.sum((st.b - rho_in) * phi)),
        "self": -st.e_self,
        "corr": st.e_c,
        "entropy": entropy_term(g, sys.kT),
    }
    t["free"] = sum(t.values())
    return t


def kerker(sys, r: np.ndarray, q0: float) -> np.ndarray:
    """P r with P = (-Lap_h)(-Lap_h + q0^2)^-1: the discrete Laplacian is
    diagonal in the Fourier basis (eigenvalues S(k) <= 0 of the FD symbol),
    so P scales each Fourier component by -S / (-S + q0^2); the constant
    component is removed."""
    nx, ny, nz = sys.n
    lam = -electrostatics.fd_symbol_3d(sys)
    rh = np.fft.fftn(r.reshape(nz, ny, nx))
    rh *= lam / (lam + q0 * q0)
    rh[0, 0, 0] = 0.0
    return np.real(np.fft.ifftn(rh)).reshape(-1)


def mix(rho_in, rho_out, beta, sys=None, kerker_q0: float = 0.0):
    d = rho_out - rho_in
    if kerker_q0 > 0.0:
        d = kerker(sys, d, kerker_q0)
    return rho_in + beta * d


class PeriodicPulay:
    """Periodic Pulay mixing (the SCF accelerator of Sec. 2.1): with
    x_k = rho_in and f_k = rho_out - rho_in, keep the last `m` differences
    dX = x_j - x_{j-1}, dF = f_j - f_{j-1}.  Every `period`-th iteration
    (k + 1 divisible by `period`, once there is history) take the
    least-squares combination
        gamma = argmin || f_k - dF gamma ||,
        x_bar = x_k - dX gamma,   f_bar = f_k - dF gamma,
        x_{k+1} = x_bar + beta P f_bar;
    otherwise the linear step x_{k+1} = x_k + beta P f_k.  P is the optional
    Kerker-type preconditioner (identity when q0 = 0).

    restart: the restarted variant the paper uses; the paper does not spell
    out the rule, and here the history is discarded after a Pulay step that
    used a full history of m pairs (the next pair is formed from x_k, f_k)."""

    def __init__(self, m: int, period: int, beta: float, sys=None, kerker_q0: float = 0.0,
                 restart: bool = False, precondition=None):
        self.m, self.period, self.beta, self.restart = m, period, beta, restart
        self.sys, self.q0 = sys, kerker_q0
        self.precondition = precondition   # optional callable in place of the Kerker step
        self.dX, self.dF = [], []
        self.x_prev = self.f_prev = None
        self.k = 0
        self.last = None   # (dF, dX, gamma) of the latest Pulay step, for diagnostics

    def _precondition(self, f):
        if self.precondition is not None:
            return self.precondition(f)
        return kerker(self.sys, f, self.q0) if self.q0 > 0.0 else f

    def step(self, x, f):
        if self.x_prev is not None and self.m > 0:
            self.dX.append(x - self.x_prev)
            self.dF.append(f - self.f_prev)
            if len(self.dX) > self.m:
                self.dX.pop(0)
                self.dF.pop(0)
        self.x_prev, self.f_prev = x.copy(), f.copy()
        pulay = self.m > 0 and len(self.dF) > 0 and (self.k + 1) % self.period == 0
        self.k += 1
        self.last = None
        if not pulay:
            return x + self.beta * self._precondition(f)
        F = np.stack(self.dF, axis=1)
        Xd = np.stack(self.dX, axis=1)
        gamma = np.linalg.solve(F.T @ F, F.T @ f)
        self.last = (F, Xd, gamma)
        xb = x - Xd @ gamma
        fb = f - F @ gamma
        if self.restart and len(self.dF) == self.m:
            self.dX, self.dF = [], []
        return xb + self.beta * self._precondition(fb)


@dataclass
class SCFResult:
    X: np.ndarray
    lam: np.ndarray
    g: np.ndarray
    mu: float
    rho_in: np.ndarray
    rho_out: np.ndarray
    history: list = field(default_factory=list)


def scf(sys, X0: np.ndarray, rho0: np.ndarray = None, max_iter: int = 50, tol: float = 1e-10,
        st: Setup = None, n_first: int = None, degree: int = None, beta: float = None,
        callback=None) -> SCFResult:
    """Run the SCF iteration from orbitals X0 (rows) and density rho0 (SAD
    if None).

    Schedule (one iteration):
      1. V_eff from rho_in (Poisson + LDA);  (lo, hi) = spectrum bounds.
      2. First iteration only: Rayleigh-Ritz of X0 gives the Ritz values that
         set the filter cut a = max Ritz value, and a0 = lo.
      3. n_first passes (first iteration) or one pass of
         filter(X, m, a, hi, a0) -> Rayleigh-Ritz, after each of which
         a = max Ritz value and a0 = min Ritz value.
      4. Occupations, rho_out, Harris-Foulkes free energy at rho_in,
         residual ||rho_out - rho_in|| / ||rho_out||, then linear mixing, or
         periodic Pulay mixing when ``sys.pulay_history`` > 0.
    Stops after the iteration whose residual is below ``tol``.
    Parity unpinned: away from the fixed point only GPU <-> oracle agreement
    is checked."""
    st = st or setup(sys)
    n_first = sys.n_first if n_first is None else n_first
    m = sys.cheb_degree if degree is None else degree
    beta = sys.mix_beta if beta is None else beta
    rho_in = atoms.sad_density(sys) if rho0 is None else rho0.copy()
    X = X0.copy()
    a = a0 = None
    pulay = None
    if getattr(sys, "pulay_history", 0) > 0:
        pulay = PeriodicPulay(sys.pulay_history, sys.pulay_period, beta, sys, getattr(sys, "kerker_q0", 0.0),
                              bool(getattr(sys, "pulay_restart", 0)))
    hist = []
    res = None
    for it in range(max_iter):
        phi, exc, vxc, veff = potential(sys, st, rho_in)
        lo, hi = hamiltonian.spectrum_bounds(sys, veff, st.projs)
        if it == 0:
            X, lam = chefsi.rayleigh_ritz(sys, veff, st.projs, X)
            a, a0 = float(lam[-1]), lo
        npass = n_first if it == 0 else 1
        for _ in range(npass):
            Y = chefsi.chebyshev_filter(sys, veff, st.projs, X, m, a, hi, a0)
            X, lam = chefsi.rayleigh_ritz(sys, veff, st.projs, Y)
            a, a0 = float(lam[-1]), float(lam[0])
        mu, g = occupations(lam, sys.n_electrons, sys.kT)
        rho_out = density(X, g)
        terms = energy_terms(sys, st, rho_in, phi, exc, vxc, lam, g)
        res = float(np.linalg.norm(rho_out - rho_in) / np.linalg.norm(rho_out))
        rec = dict(it=it, residual=res, mu=mu, lam=lam.copy(), bounds=(a, hi, a0), **terms)
        hist.append(rec)
        if callback is not None:
            callback(rec)
        rho_prev = rho_in
        if pulay is not None:
            rho_in = pulay.step(rho_in, rho_out - rho_in)
        else:
            rho_in = mix(rho_in, rho_out, beta, sys, getattr(sys, "kerker_q0", 0.0))
        if res < tol:
            break
    return SCFResult(X=X, lam=lam, g=g, mu=mu, rho_in=rho_prev, rho_out=rho_out, history=hist)


# ---------------------------------------------------------------- spin
# Spin-polarised form (eq. (1)-(2) with a spin index): one orbital block per
# spin with H_s = -1/2 Lap + phi + v_xc^s + V_nl; occupations f_n^s (one
# electron per state) with a common Fermi level, sum_s sum_n f_n^s = N_e;
# rho^s = sum_n f_n^s |psi_n^s|^2; phi from the total density.  Sec. 2.1:
# the mixing acts on the vector of both spin densities at once.


def occupations_spin(lam_up, lam_dn, n_electrons: float, kT: float, tol: float = 1e-13, max_iter: int = 500):
    """Common mu over both spins by bisection (one electron per state);
    returns (mu, f_up, f_dn)."""
    lam = np.concatenate([np.asarray(lam_up, dtype=np.float64), np.asarray(lam_dn, dtype=np.float64)])
    if n_electrons > lam.size or n_electrons <= 0.0:
        raise FermiError("electron count outside (0, N_up + N_dn]")
    lo = float(lam.min()) - 40.0 * kT
    hi = float(lam.max()) + 40.0 * kT
    mu = 0.5 * (lo + hi)
    for _ in range(max_iter):
        mu = 0.5 * (lo + hi)
        n = float(np.sum(fermi(lam, mu, kT)))
        if abs(n - n_electrons) < tol:
            break
        if n < n_electrons:
            lo = mu
        else:
            hi = mu
        if not (lo < 0.5 * (lo + hi) < hi):
            break
    f = fermi(lam, mu, kT)
    return mu, f[:len(lam_up)], f[len(lam_up):]


def entropy_term_spin(f, kT):
    """kT sum [f ln f + (1-f) ln(1-f)] over spin states (0 ln 0 = 0)."""
    s = 0.0
    for v in np.asarray(f):
        if 0.0 < v < 1.0:
            s += v * np.log(v) + (1.0 - v) * np.log(1.0 - v)
    return kT * s


def potential_spin(sys, st: Setup, rho_up: np.ndarray, rho_dn: np.ndarray):
    """(phi, eps_xc, v_xc_up, v_xc_dn, V_eff_up, V_eff_dn)."""
    phi = electrostatics.hartree_ionic_potential(sys, rho_up + rho_dn, st.b)
    exc, vu, vd = xc.lsda(rho_up, rho_dn, sys.rho_floor)
    return phi, exc, vu, vd, phi + vu, phi + vd


def energy_terms_spin(sys, st: Setup, rho_up, rho_dn, phi, exc, vu, vd, lam_up, lam_dn, f_up, f_dn):
    """Harris-Foulkes free energy at the input spin densities (the spin form
    of ``energy_terms``)."""
    dV = sys.dV
    rho = rho_up + rho_dn
    t = {
        "band": float(np.sum(f_up * lam_up) + np.sum(f_dn * lam_dn)),
        "exc": dV * float(np.sum(rho * exc)),
        "vxc_dc": -dV * float(np.sum(rho_up * vu + rho_dn * vd)),
        "elec": 0.5 * dV * float(np.sum((st.b - rho) * phi)),
        "self": -st.e_self,
        "corr": st.e_c,
        "entropy": entropy_term_spin(np.concatenate([f_up, f_dn]), sys.kT),
    }
    t["free"] = sum(t.values())
    return t


def spin_precondition(sys, f: np.ndarray, q0: float) -> np.ndarray:
    """Preconditioner of the spin mixing vector [f_up; f_dn]: the Kerker step
    acts on the total f_up + f_dn, the magnetisation part f_up - f_dn is
    passed unchanged (filtering each spin separately would remove the
    constant mode of the magnetisation and freeze the total moment)."""
    if not q0 > 0.0:
        return f
    nd = sys.nd
    t = kerker(sys, f[:nd] + f[nd:], q0)
    m = f[:nd] - f[nd:]
    return np.concatenate([0.5 * (t + m), 0.5 * (t - m)])


def sad_density_spin(sys):
    """Atomic-density guess split by the starting polarisation zeta0 =
    sys.spin_zeta0: rho_up = (1 + zeta0) rho / 2, rho_dn = (1 - zeta0) rho / 2."""
    rho = atoms.sad_density(sys)
    z = float(getattr(sys, "spin_zeta0", 0.0))
    return 0.5 * (1.0 + z) * rho, 0.5 * (1.0 - z) * rho


@dataclass
class SpinSCFResult:
    X: tuple
    lam: tuple
    f: tuple
    mu: float
    rho_in: np.ndarray      # [rho_up; rho_dn] of the last iteration
    rho_out: np.ndarray
    history: list


def scf_spin(sys, X0_up: np.ndarray, X0_dn: np.ndarray, rho0: np.ndarray = None, max_iter: int = 50,
             tol: float = 1e-10, st: Setup = None, n_first: int = None, degree: int = None,
             beta: float = None) -> SpinSCFResult:
    """The SCF schedule of ``scf`` for the spin-polarised form: per spin the
    filter bounds and passes are those of ``scf`` with that spin's V_eff and
    block; occupations with a common mu; residual and mixing over
    [rho_up; rho_dn] (linear, or periodic Pulay when sys.pulay_history > 0,
    with ``spin_precondition``).  rho0: [rho_up; rho_dn] or None (split SAD).
    Parity unpinned away from the fixed point, as for ``scf``."""
    st = st or setup(sys)
    n_first = sys.n_first if n_first is None else n_first
    m = sys.cheb_degree if degree is None else degree
    beta = sys.mix_beta if beta is None else beta
    nd = sys.nd
    q0 = getattr(sys, "kerker_q0", 0.0)
    if rho0 is None:
        ru, rd = sad_density_spin(sys)
        x = np.concatenate([ru, rd])
    else:
        x = np.array(rho0, dtype=np.float64)
    Xs = [X0_up.copy(), X0_dn.copy()]
    ab = [None, None]
    pulay = None
    if getattr(sys, "pulay_history", 0) > 0:
        pulay = PeriodicPulay(sys.pulay_history, sys.pulay_period, beta, restart=bool(getattr(sys, "pulay_restart", 0)),
                              precondition=lambda f: spin_precondition(sys, f, q0))
    hist = []
    lams = [None, None]
    for it in range(max_iter):
        phi, exc, vu, vd, veu, ved = potential_spin(sys, st, x[:nd], x[nd:])
        for s, veff in enumerate((veu, ved)):
            lo, hi = hamiltonian.spectrum_bounds(sys, veff, st.projs)
            if it == 0:
                Xs[s], lam = chefsi.rayleigh_ritz(sys, veff, st.projs, Xs[s])
                a, a0 = float(lam[-1]), lo
            else:
                a, a0 = ab[s]
            npass = n_first if it == 0 else 1
            for _ in range(npass):
                Y = chefsi.chebyshev_filter(sys, veff, st.projs, Xs[s], m, a, hi, a0)
                Xs[s], lam = chefsi.rayleigh_ritz(sys, veff, st.projs, Y)
                a, a0 = float(lam[-1]), float(lam[0])
            ab[s] = (a, a0)
            lams[s] = lam
        mu, fu, fd = occupations_spin(lams[0], lams[1], sys.n_electrons, sys.kT)
        rho_out = np.concatenate([density(Xs[0], fu), density(Xs[1], fd)])
        terms = energy_terms_spin(sys, st, x[:nd], x[nd:], phi, exc, vu, vd, lams[0], lams[1], fu, fd)
        res = float(np.linalg.norm(rho_out - x) / np.linalg.norm(rho_out))
        mag = sys.dV * float(np.sum(rho_out[:nd] - rho_out[nd:]))
        rec = dict(it=it, residual=res, mu=mu, lam=(lams[0].copy(), lams[1].copy()), magnetization=mag, **terms)
        hist.append(rec)
        x_prev = x
        if pulay is not None:
            x = pulay.step(x, rho_out - x)
        else:
            x = x + beta * spin_precondition(sys, rho_out - x, q0)
        if res < tol:
            break
    return SpinSCFResult(X=tuple(Xs), lam=tuple(lams), f=(fu, fd), mu=mu, rho_in=x_prev, rho_out=rho_out,
                         history=hist)
