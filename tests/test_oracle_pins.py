"""Pins of the CPU oracle against facts fixed by mathematics and by the paper's
discretisation (Sec. 2.1), independent of the oracle's own formulas.

Each test is chosen so that a plausible slip in the oracle (a dropped term, a
sign, a transposed index, a wrong weight) fails it.
"""
from fractions import Fraction
from math import erf, log, pi, sqrt

import numpy as np
import pytest
from numpy.polynomial import chebyshev as npcheb
from scipy.optimize import brentq

import workloads as W
from oracle import atoms, chefsi, electrostatics, fd, hamiltonian, scf, xc


# ---------------------------------------------------------------- FD stencil

def test_fd_weights_exact_on_polynomials():
    """The 12th-order centred stencil is exact for x^k, k <= 13, and not for
    k = 14 (moment conditions fix all seven weights)."""
    n_o = 6
    w = fd.fd_weights_exact(n_o)
    x = Fraction(3, 7)
    h = Fraction(1, 5)
    for k in range(0, 16):
        f = lambda t: t ** k
        approx = w[0] * f(x)
        for q in range(1, n_o + 1):
            approx += w[q] * (f(x + q * h) + f(x - q * h))
        approx /= h * h
        exact = k * (k - 1) * x ** (k - 2) if k >= 2 else Fraction(0)
        if k <= 13:
            assert approx == exact, k
        else:
            assert approx != exact, k


def test_fd_weights_low_orders():
    """Half-order 1 and 2 give the textbook 3- and 5-point stencils."""
    assert fd.fd_weights_exact(1) == [Fraction(-2), Fraction(1)]
    assert fd.fd_weights_exact(2) == [Fraction(-5, 2), Fraction(4, 3), Fraction(-1, 12)]


def test_symbol_minimum_at_pi_and_small_theta():
    th = np.linspace(0, np.pi, 20001)
    s = fd.symbol(th, 6)
    assert np.argmin(s) == th.size - 1
    assert np.all(np.diff(s) < 0)
    t = np.array([1e-3, 1e-2, 0.1])
    # 12th order: s(theta) = -theta^2 + O(theta^14)
    np.testing.assert_allclose(fd.symbol(t, 6), -t * t, rtol=0, atol=1e-13)


def test_laplacian_plane_wave_continuum():
    """On a smooth periodic plane wave the discrete Laplacian matches the
    continuum -|k|^2 to the stencil's order."""
    s = W.config1(0)
    nx, ny, nz = s.n
    hx, hy, hz = s.h
    z, y, x = np.meshgrid(np.arange(nz) * hz, np.arange(ny) * hy, np.arange(nx) * hx, indexing="ij")
    k = 2 * np.pi * np.array([1, 2, 1]) / np.array(s.L)
    f = np.cos(k[0] * x + k[1] * y + k[2] * z)
    lap = fd.laplacian(f, s.h, 6)
    np.testing.assert_allclose(lap, -np.dot(k, k) * f, atol=1e-9)


# ---------------------------------------------------------------- Hamiltonian

def _free(sys):
    return np.zeros(sys.nd)


def test_free_electron_closed_form_plane_waves():
    """V_eff = 0, no nonlocal: plane waves are eigenvectors with eigenvalue
    -1/2 sum_d s(2 pi j_d / N_d) / h_d^2 (closed form of the discrete
    Laplacian); on the config-1 grid the first shell equals 1/2 (2 pi / 8)^2
    to 1e-12."""
    s = W.config1(0)
    nx, ny, nz = s.n
    hx, hy, hz = s.h
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    for j in [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (2, 1, 3), (5, 0, 7)]:
        th = [2 * np.pi * j[0] / nx, 2 * np.pi * j[1] / ny, 2 * np.pi * j[2] / nz]
        lam = -0.5 * sum(fd.symbol(t, 6) / hd ** 2 for t, hd in zip(th, (hx, hy, hz)))
        for fn in (np.cos, np.sin):
            v = fn(th[0] * ix + th[1] * iy + th[2] * iz).reshape(1, -1)
            Hv = hamiltonian.apply_H(s, _free(s), [], v)
            np.testing.assert_allclose(Hv, lam * v, atol=1e-12 * max(1.0, lam))
    lam1 = -0.5 * fd.symbol(2 * np.pi / 24, 6) / (1.0 / 3.0) ** 2
    assert abs(lam1 - 0.5 * (2 * np.pi / 8) ** 2) < 1e-12


def test_dense_free_electron_spectrum():
    """Brute force: the dense H of a tiny non-cubic grid with V = 0 has exactly
    the closed-form spectrum {-1/2 sum_d s(theta_d)/h_d^2}."""
    s = W.tiny_system(n=(8, 9, 10), L=(2.4, 2.7, 3.1), with_nonlocal=False)
    H = hamiltonian.dense_H(s, _free(s), [])
    ev = np.linalg.eigvalsh(0.5 * (H + H.T))
    nx, ny, nz = s.n
    hx, hy, hz = s.h
    sx = fd.symbol(2 * np.pi * np.arange(nx) / nx, 6) / hx ** 2
    sy = fd.symbol(2 * np.pi * np.arange(ny) / ny, 6) / hy ** 2
    sz = fd.symbol(2 * np.pi * np.arange(nz) / nz, 6) / hz ** 2
    closed = np.sort((-0.5 * (sz[:, None, None] + sy[None, :, None] + sx[None, None, :])).ravel())
    np.testing.assert_allclose(ev, closed, atol=1e-10)


def test_constant_potential_shift():
    s = W.tiny_system(n=(8, 9, 10), L=(2.4, 2.7, 3.1))
    projs = atoms.projectors(s)
    rng = np.random.default_rng(1)
    X = rng.standard_normal((3, s.nd))
    v = rng.standard_normal(s.nd)
    c = 0.731
    d = hamiltonian.apply_H(s, v + c, projs, X) - hamiltonian.apply_H(s, v, projs, X)
    np.testing.assert_allclose(d, c * X, atol=1e-12)


def test_hermiticity_with_nonlocal():
    s = W.tiny_system()
    projs = atoms.projectors(s)
    rng = np.random.default_rng(2)
    v = rng.standard_normal(s.nd)
    X = rng.standard_normal((4, s.nd))
    Y = rng.standard_normal((4, s.nd))
    a = Y @ hamiltonian.apply_H(s, v, projs, X).T
    b = hamiltonian.apply_H(s, v, projs, Y) @ X.T
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(a))


def test_nonlocal_single_atom_on_grid_point():
    """One atom on a grid point: chi_s is even and the chi_p are odd about it,
    so dV chi chi^T has eigenvalues gamma_l dV ||chi_lm||^2, and continuum
    normalisation makes dV ||chi_lm||^2 = 1 up to quadrature/cut-off error."""
    s = W.tiny_system(n=(26, 26, 26), L=(7.8, 7.8, 7.8), n_atoms=1)
    s.pos = np.array([s.h]) * 13.0
    s.rc_nl = 0.9
    s.rcut_nl = 2.75          # not a grid distance, so the cut keeps the symmetry
    s.gamma = np.array([[0.37, -0.81]])
    projs = atoms.projectors(s)
    P = projs[0]
    G = s.dV * (P.chi @ P.chi.T)           # Gram of the four projectors
    np.testing.assert_allclose(G - np.diag(np.diag(G)), 0.0, atol=1e-14)
    np.testing.assert_allclose(np.diag(G), 1.0, atol=2e-4)
    # eigenvalues of the nonlocal operator restricted to the support
    Xs = np.eye(s.nd)[P.idx]
    V = hamiltonian.apply_H(s, np.zeros(s.nd), projs, Xs)[:, P.idx] - \
        hamiltonian.apply_H(s, np.zeros(s.nd), [], Xs)[:, P.idx]
    ev = np.linalg.eigvalsh(0.5 * (V + V.T))
    nz = ev[np.abs(ev) > 1e-10]
    expect = np.sort(np.array([0.37, -0.81, -0.81, -0.81]) * np.diag(G))
    np.testing.assert_allclose(np.sort(nz), expect, atol=1e-12)


def test_spectrum_bounds_enclose_dense_spectrum():
    s = W.tiny_system(n=(9, 10, 11), L=(2.7, 3.0, 3.3))
    projs = atoms.projectors(s)
    v = np.random.default_rng(4).uniform(-1, 1, s.nd)
    lo, hi = hamiltonian.spectrum_bounds(s, v, projs)
    ev = np.linalg.eigvalsh(hamiltonian.dense_H(s, v, projs))
    assert lo <= ev[0] and ev[-1] <= hi


# ---------------------------------------------------------------- atoms

def test_pseudocharge_and_sad_normalisation():
    for s in (W.config1(0), W.tiny_system()):
        b = atoms.pseudocharge(s)
        assert abs(s.dV * b.sum() + s.Z.sum()) < 1e-11
        rho0 = atoms.sad_density(s)
        assert abs(s.dV * rho0.sum() - s.n_electrons) < 1e-11
        assert rho0.min() > 0


def test_self_energy_closed_form():
    """Self-energy of a Gaussian charge Z of width rc: Z^2 / (sqrt(2 pi) rc)."""
    s = W.config1(0)
    e = atoms.self_energy(s)
    closed = s.n_atoms * s.Z[0] ** 2 / (sqrt(2 * pi) * s.rc_loc[0])
    assert abs(e - closed) < 1e-10


def test_overlap_correction_invariances():
    s = W.config1(0)
    e0 = atoms.overlap_correction(s)
    s2 = W.config1(0)
    s2.pos = np.mod(s.pos + np.array([0.37, -1.2, 2.9]), 8.0)
    assert abs(atoms.overlap_correction(s2) - e0) < 1e-12
    # a single pair far apart in a big cell: erfc(d/s)/d by hand
    t = W.tiny_system(n=(13, 13, 13), L=(40.0, 40.0, 40.0), with_nonlocal=False)
    t.pos = np.array([[1.0, 1.0, 1.0], [2.5, 1.0, 1.0]])
    from math import erfc
    ref = t.Z[0] * t.Z[1] * erfc(1.5 / sqrt(2 * 0.8 ** 2)) / 1.5
    assert abs(atoms.overlap_correction(t) - ref) < 1e-14


# ---------------------------------------------------------------- Poisson

def test_poisson_solution_satisfies_stencil_equation():
    """The FFT solve and the real-space stencil are different routes to the
    same operator: -Delta_h phi must equal 4 pi (r - mean r)."""
    s = W.tiny_system(n=(13, 14, 15), L=(4.0, 4.3, 4.6))
    r = np.random.default_rng(5).standard_normal(s.nd)
    phi = electrostatics.solve_poisson(s, r)
    lap = fd.laplacian(phi.reshape(s.n[2], s.n[1], s.n[0]), s.h, 6).ravel()
    np.testing.assert_allclose(-lap, 4 * np.pi * (r - r.mean()), atol=1e-10)
    assert abs(phi.mean()) < 1e-13


def test_kerker_preconditioner_solves_screened_stencil_equation():
    """y = P r must satisfy (-Delta_h + q0^2) y = -Delta_h r, with Delta_h
    applied by the real-space stencil (a different route from the Fourier
    scaling); P removes the mean and tends to r - mean(r) as q0 -> 0."""
    s = W.tiny_system(n=(13, 14, 15), L=(4.0, 4.3, 4.6))
    r = np.random.default_rng(6).standard_normal(s.nd)
    shape = (s.n[2], s.n[1], s.n[0])
    for q0 in (0.5, 1.0, 2.5):
        y = scf.kerker(s, r, q0)
        lap_y = fd.laplacian(y.reshape(shape), s.h, 6).ravel()
        lap_r = fd.laplacian(r.reshape(shape), s.h, 6).ravel()
        np.testing.assert_allclose(-lap_y + q0 * q0 * y, -lap_r, atol=1e-10)
        assert abs(y.mean()) < 1e-14
    np.testing.assert_allclose(scf.kerker(s, r, 1e-7), r - r.mean(), atol=1e-10)


def test_kerker_mixing_conserves_electrons():
    s = W.tiny_system(n=(13, 14, 15), L=(4.0, 4.3, 4.6))
    rng = np.random.default_rng(7)
    rin = rng.uniform(0.1, 1.0, s.nd)
    rout = rng.uniform(0.1, 1.0, s.nd)
    rout *= rin.sum() / rout.sum()
    new = scf.mix(rin, rout, 0.3, s, 1.0)
    assert abs(new.sum() - rin.sum()) <= 1e-10 * rin.sum()
    np.testing.assert_allclose(scf.mix(rin, rout, 0.3), rin + 0.3 * (rout - rin), rtol=0, atol=0)


def test_poisson_plane_wave_continuum():
    s = W.config1(0)
    nx, ny, nz = s.n
    hx, hy, hz = s.h
    z, y, x = np.meshgrid(np.arange(nz) * hz, np.arange(ny) * hy, np.arange(nx) * hx, indexing="ij")
    k = 2 * np.pi * np.array([1, 0, 2]) / 8.0
    r = np.sin(k[0] * x + k[2] * z).ravel()
    phi = electrostatics.solve_poisson(s, r)
    np.testing.assert_allclose(phi, 4 * np.pi / np.dot(k, k) * r, atol=1e-10)


# ---------------------------------------------------------------- XC

def test_slater_exchange_closed_form():
    # uniform gas at r_s = 1: eps_x = -(3/4)(9/(4 pi^2))^(1/3) ... via rho
    rho = 3.0 / (4.0 * pi)          # r_s = 1
    ex, vx = xc.slater_exchange(np.array([rho]))
    assert abs(ex[0] - (-0.75 * (9.0 / (4.0 * pi * pi)) ** (1.0 / 3.0))) < 1e-15
    assert abs(ex[0] - (-0.458165293283143)) < 1e-12


def test_pw92_high_density_coefficient():
    """The log coefficient of eps_c as r_s -> 0 is (1 - ln 2)/pi^2."""
    assert abs(xc.PW92_A - (1 - log(2)) / pi ** 2) < 1e-6
    r1, r2 = 1e-8, 1e-9
    e1, _ = xc.pw92_correlation(np.array([r1]))
    e2, _ = xc.pw92_correlation(np.array([r2]))
    slope = (e1[0] - e2[0]) / (log(r1) - log(r2))
    assert abs(slope - xc.PW92_A) < 1e-4


def sqrt_rs_coefficient(G_of_rs, A):
    """Coefficient c of r_s^(1/2) in G(r_s) = A ln r_s + const + c r_s^(1/2)
    + O(r_s ln r_s), from two points r and 4r at r = 1e-14, where the
    O(r_s ln r_s) remainder changes by less than 1e-6 of the r_s^(1/2) term
    of a fit whose b2 is off by a quarter percent."""
    r1, r2 = 1e-14, 4e-14
    g1, g2 = G_of_rs(r1) - A * log(r1), G_of_rs(r2) - A * log(r2)
    return (g2 - g1) / (sqrt(r2) - sqrt(r1))


def test_pw92_fit_has_no_sqrt_rs_term():
    """The exact high-density expansion of the correlation energy is
    A ln r_s - c1 + O(r_s ln r_s): it has no r_s^(1/2) term.  Expanding
    ln(1 + 1/Q1) with Q1 = 2A (b1 r_s^(1/2) + b2 r_s + ...) gives that term
    the coefficient -2A (2A b1 - b2/b1), which vanishes iff b2 = 2 A b1^2.
    Checked on the constants and numerically on the oracle's function, so a
    typo in b1 or b2 (a quarter percent moves the coefficient 300-fold past
    the bar) fails."""
    b1, b2 = xc.PW92_BETA[0], xc.PW92_BETA[1]
    assert abs(b2 - 2.0 * xc.PW92_A * b1 * b1) / b2 < 1e-4
    coef = sqrt_rs_coefficient(lambda r: xc.pw92_correlation(np.array([r]))[0][0], xc.PW92_A)
    scale = 2.0 * xc.PW92_A * (2.0 * xc.PW92_A * b1)   # either half of the cancelling pair
    assert abs(coef) < 2e-4 * scale, coef


def test_vxc_is_derivative_of_energy_density():
    rho = np.array([1e-4, 3e-3, 0.02, 0.1, 0.7, 3.0])
    eps, v = xc.lda(rho)
    d = 1e-6 * rho
    ep, _ = xc.lda(rho + d)
    em, _ = xc.lda(rho - d)
    num = ((rho + d) * ep - (rho - d) * em) / (2 * d)
    np.testing.assert_allclose(v, num, rtol=1e-8)


def test_pw92_derivative():
    rs = np.array([0.3, 1.0, 2.0, 5.0, 20.0])
    ec, dec = xc.pw92_correlation(rs)
    d = 1e-6 * rs
    num = (xc.pw92_correlation(rs + d)[0] - xc.pw92_correlation(rs - d)[0]) / (2 * d)
    np.testing.assert_allclose(dec, num, rtol=1e-7)
    assert np.all(ec < 0)


# ---------------------------------------------------------------- filter / RR

def _tiny_dense(seed=6):
    s = W.tiny_system(n=(9, 10, 11), L=(2.9, 3.2, 3.5), n_states=6)
    projs = atoms.projectors(s)
    v = np.random.default_rng(seed).uniform(-0.5, 0.5, s.nd)
    H = hamiltonian.dense_H(s, v, projs)
    ev, U = np.linalg.eigh(0.5 * (H + H.T))
    return s, projs, v, ev, U


def test_filter_on_eigenvectors_is_scaled_chebyshev():
    """p_m(lam) = T_m((lam - c)/e) / T_m((a0 - c)/e), evaluated with NumPy's
    Chebyshev series rather than the recurrence."""
    s, projs, v, ev, U = _tiny_dense()
    idx = [0, 3, 50, 400, ev.size - 1]
    X = U[:, idx].T
    a, b, a0 = ev[40], ev[-1] + 0.1, ev[0] - 0.05
    m = 9
    Y = chefsi.chebyshev_filter(s, v, projs, X, m, a, b, a0)
    e, c = (b - a) / 2, (b + a) / 2
    Tm = lambda t: npcheb.chebval(t, [0] * m + [1])
    for r, j in enumerate(idx):
        p = Tm((ev[j] - c) / e) / Tm((a0 - c) / e)
        np.testing.assert_allclose(Y[r], p * X[r], atol=1e-11 * max(1, abs(p)))


def test_rayleigh_ritz_brute_force():
    """CheFSI at fixed V_eff, iterated, reproduces the lowest N_s eigenvalues
    of the dense H to 1e-9 Ha."""
    s, projs, v, ev, U = _tiny_dense()
    ns = s.n_states
    X = W.initial_orbitals(s.nd, ns, 0)
    X, lam = chefsi.rayleigh_ritz(s, v, projs, X)
    lo, hi = hamiltonian.spectrum_bounds(s, v, projs)
    a, a0 = lam[-1], lo
    for _ in range(40):
        Y = chefsi.chebyshev_filter(s, v, projs, X, 10, a, hi, a0)
        X, lam = chefsi.rayleigh_ritz(s, v, projs, Y)
        a, a0 = lam[-1], lam[0]
    np.testing.assert_allclose(lam[:ns - 1], ev[:ns - 1], atol=1e-9)
    O = s.dV * X @ X.T
    assert np.max(np.abs(O - np.eye(ns))) < 1e-13
    # eigen-residual of the converged Ritz pairs
    R = hamiltonian.apply_H(s, v, projs, X) - lam[:, None] * X
    assert np.max(np.abs(R[:ns - 1])) < 1e-6


def test_orthonormalize_rejects_rank_deficient():
    s = W.tiny_system()
    Y = W.initial_orbitals(s.nd, 3, 0)
    Y[2] = Y[1]
    with pytest.raises(chefsi.NotSPD):
        chefsi.orthonormalize(s, Y)


# ---------------------------------------------------------------- occupations / energy

def test_occupations_against_library_root_finder():
    lam = np.sort(np.random.default_rng(7).uniform(-0.6, 0.4, 12))
    mu, g = scf.occupations(lam, 16.0, 0.01)
    f = lambda m: 2 * np.sum(1 / (1 + np.exp((lam - m) / 0.01))) - 16.0
    mu_ref = brentq(f, lam[0] - 1, lam[-1] + 1, xtol=1e-15)
    assert abs(mu - mu_ref) < 1e-11
    assert abs(g.sum() - 16.0) < 1e-12
    with pytest.raises(scf.FermiError):
        scf.occupations(lam, 25.0, 0.01)


def test_fermi_no_overflow():
    f = scf.fermi(np.array([-1e4, 0.0, 1e4]), 0.0, 0.01)
    np.testing.assert_array_equal(f, [1.0, 0.5, 0.0])


@pytest.fixture(scope="module")
def cfg1_converged():
    s = W.config1(0)
    st = scf.setup(s)
    X0 = W.initial_orbitals(s.nd, s.n_states, 0)
    r = scf.scf(s, X0, max_iter=80, tol=1e-10, st=st)
    return s, st, r


def test_density_electron_count(cfg1_converged):
    s, st, r = cfg1_converged
    assert abs(s.dV * r.rho_out.sum() - s.n_electrons) < 1e-11
    assert abs(r.g.sum() - s.n_electrons) < 1e-12


def test_energy_gauge_invariance(cfg1_converged):
    """phi -> phi + 1 shifts every eigenvalue by +1; the free energy must not
    change (needs dV sum b = -N_e and the signs of every term right)."""
    s, st, r = cfg1_converged
    rho = r.rho_in
    phi, exc, vxc, veff = scf.potential(s, st, rho)
    t0 = scf.energy_terms(s, st, rho, phi, exc, vxc, r.lam, r.g)
    t1 = scf.energy_terms(s, st, rho, phi + 1.0, exc, vxc, r.lam + 1.0, r.g)
    assert abs(t0["free"] - t1["free"]) < 1e-10


def test_scf_fixed_point_and_dense_eigenvalues(cfg1_converged):
    """At convergence rho_out(rho_in) = rho_in and the Ritz values are the
    lowest eigenvalues of the dense-free check H[rho_in] (filtered to
    convergence at fixed V_eff)."""
    s, st, r = cfg1_converged
    assert r.history[-1]["residual"] < 1e-10
    phi, exc, vxc, veff = scf.potential(s, st, r.rho_in)
    R = hamiltonian.apply_H(s, veff, st.projs, r.X) - r.lam[:, None] * r.X
    # occupied states are converged eigenpairs of H[rho_in]
    occ = r.g > 1e-6
    assert np.max(np.abs(R[occ])) < 1e-5


def test_scf_fixed_point_independent_of_start():
    """The converged density and energy do not depend on the random X0."""
    s = W.config1(0)
    st = scf.setup(s)
    ra = scf.scf(s, W.initial_orbitals(s.nd, s.n_states, 0), max_iter=80, tol=1e-9, st=st)
    rb = scf.scf(s, W.initial_orbitals(s.nd, s.n_states, 5), max_iter=80, tol=1e-9, st=st)
    fa, fb = ra.history[-1]["free"], rb.history[-1]["free"]
    assert abs(fa - fb) / s.n_atoms < 1e-9
    np.testing.assert_allclose(ra.lam[:8], rb.lam[:8], atol=1e-7)


# ---------------------------------------------------------------- Pulay mixing

def test_pulay_solves_linear_fixed_point_in_dim_plus_one_steps():
    """On a linear map x -> A x + b of dimension n, Pulay (Anderson)
    extrapolation at every step with history >= n reaches the fixed point
    after n + 1 steps (the residuals span the Krylov space)."""
    rng = np.random.default_rng(11)
    n = 6
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = (Q * rng.uniform(-0.9, 0.9, n)) @ Q.T
    b = rng.standard_normal(n)
    xstar = np.linalg.solve(np.eye(n) - A, b)
    mixer = scf.PeriodicPulay(m=n, period=1, beta=0.5)
    x = np.zeros(n)
    for _ in range(n + 2):
        x = mixer.step(x, A @ x + b - x)
    assert np.linalg.norm(x - xstar) <= 1e-9 * np.linalg.norm(xstar)
    # plain linear mixing is nowhere near after the same number of steps
    y = np.zeros(n)
    for _ in range(n + 2):
        y = y + 0.5 * (A @ y + b - y)
    assert np.linalg.norm(y - xstar) > 1e-3 * np.linalg.norm(xstar)


def test_pulay_without_history_is_linear_mixing_and_residual_is_orthogonal():
    rng = np.random.default_rng(12)
    x, f = rng.standard_normal(50), rng.standard_normal(50)
    assert np.array_equal(scf.PeriodicPulay(m=0, period=1, beta=0.3).step(x, f), x + 0.3 * f)
    mixer = scf.PeriodicPulay(m=4, period=1, beta=0.3)
    xs = [rng.standard_normal(50) for _ in range(5)]
    fs = [rng.standard_normal(50) for _ in range(5)]
    for xk, fk in zip(xs[:-1], fs[:-1]):
        mixer.step(xk, fk)
    F = np.stack([fs[j] - fs[j - 1] for j in range(1, 5)], axis=1)
    Xd = np.stack([xs[j] - xs[j - 1] for j in range(1, 5)], axis=1)
    new = mixer.step(xs[-1], fs[-1])
    gamma = np.linalg.lstsq(F, fs[-1], rcond=None)[0]
    fbar = fs[-1] - F @ gamma
    assert np.max(np.abs(F.T @ fbar)) < 1e-10
    np.testing.assert_allclose(new, xs[-1] - Xd @ gamma + 0.3 * fbar, atol=1e-12)


def test_pulay_off_period_steps_are_kerker_linear_mixing():
    """Between Pulay steps the mixer is exactly the preconditioned linear
    step; a period longer than the run leaves only those."""
    sys_ = W.tiny_system(n=(14, 14, 16))
    rng = np.random.default_rng(13)
    mixer = scf.PeriodicPulay(m=5, period=100, beta=0.3, sys=sys_, kerker_q0=1.0)
    for _ in range(4):
        x, f = rng.standard_normal(sys_.nd), rng.standard_normal(sys_.nd)
        np.testing.assert_allclose(mixer.step(x, f), scf.mix(x, x + f, 0.3, sys_, 1.0), rtol=0, atol=1e-13)


def test_pulay_single_pair_is_projection_and_restart_clears_full_history():
    """With one difference pair the least-squares weight is the projection
    <dF, f> / <dF, dF>; the restarted form forgets a full history after it
    has been used, so the step after a restart again sees exactly one pair."""
    rng = np.random.default_rng(14)
    xs = [rng.standard_normal(40) for _ in range(5)]
    fs = [rng.standard_normal(40) for _ in range(5)]
    mixer = scf.PeriodicPulay(m=2, period=1, beta=0.25, restart=True)
    out = [mixer.step(xk, fk) for xk, fk in zip(xs, fs)]

    def one_pair(k):
        dx, df = xs[k] - xs[k - 1], fs[k] - fs[k - 1]
        g = np.dot(df, fs[k]) / np.dot(df, df)
        return xs[k] - g * dx + 0.25 * (fs[k] - g * df)

    np.testing.assert_array_equal(out[0], xs[0] + 0.25 * fs[0])
    np.testing.assert_allclose(out[1], one_pair(1), atol=1e-12)
    # iteration 2 uses the pairs (1, 2) and fills the history -> restart
    assert len(mixer.dF) == 0
    np.testing.assert_allclose(out[3], one_pair(3), atol=1e-12)
    # without restart iteration 3 would have used two pairs
    keep = scf.PeriodicPulay(m=2, period=1, beta=0.25)
    out_keep = [keep.step(xk, fk) for xk, fk in zip(xs, fs)]
    assert np.max(np.abs(out_keep[3] - one_pair(3))) > 1e-3
