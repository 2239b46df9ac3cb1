"""Pins of the oracle's spin-polarised form (LSDA, common-mu occupations,
spin mixing, spin SCF) against facts it does not compute itself."""
import numpy as np
from dataclasses import replace

import workloads as W
from oracle import scf, xc


def test_lsda_equal_spins_is_lda():
    rho = np.geomspace(1e-16, 50.0, 40)
    e, v = xc.lda(rho)
    e2, vu, vd = xc.lsda(0.5 * rho, 0.5 * rho)
    np.testing.assert_allclose(e2, e, rtol=1e-14, atol=0)
    np.testing.assert_allclose(vu, v, rtol=1e-14, atol=0)
    np.testing.assert_allclose(vd, v, rtol=1e-14, atol=0)


def test_lsda_potentials_are_derivatives_of_the_energy_density():
    """v_s = d(rho eps_xc)/d rho_s by central differences, across zeta."""
    rng = np.random.default_rng(3)
    ru = rng.uniform(1e-3, 2.0, 30)
    rd = ru * rng.uniform(0.02, 1.5, 30)
    _, vu, vd = xc.lsda(ru, rd)

    def E(a, b):
        e, _, _ = xc.lsda(a, b)
        return (a + b) * e
    h = 1e-5
    dU = (E(ru * (1 + h), rd) - E(ru * (1 - h), rd)) / (2 * h * ru)
    dD = (E(ru, rd * (1 + h)) - E(ru, rd * (1 - h))) / (2 * h * rd)
    np.testing.assert_allclose(vu, dU, rtol=1e-7, atol=1e-9)
    np.testing.assert_allclose(vd, dD, rtol=1e-7, atol=1e-9)


def test_lsda_fully_polarised_limits():
    """Exchange of a fully polarised gas is 2^(1/3) times the unpolarised one
    at the same density; correlation reduces to the polarised fit; the
    interpolation function has f(0) = 0, f(1) = 1 and the curvature FZ20."""
    rho = np.array([1e-3, 0.05, 1.0, 10.0])
    ex_unpol, _ = xc.slater_exchange(rho)
    e, _, _ = xc.lsda(rho, np.zeros_like(rho), rho_floor=1e-300)
    ec1, _ = xc.pw92_G(xc.rs_of(rho), *xc.PW92_POL)
    np.testing.assert_allclose(e, 2.0 ** (1.0 / 3.0) * ex_unpol + ec1, rtol=1e-12)
    f0, _ = xc.spin_interp(np.array(0.0))
    f1, _ = xc.spin_interp(np.array(1.0))
    assert abs(f0) < 1e-15 and abs(f1 - 1.0) < 1e-15
    h = 1e-4
    fp, _ = xc.spin_interp(np.array(h))
    fm, _ = xc.spin_interp(np.array(-h))
    assert abs((fp + fm) / h ** 2 - xc.FZ20) < 1e-6
    # f' against differences of f
    z = np.array([-0.7, -0.1, 0.3, 0.9])
    _, df = xc.spin_interp(z)
    np.testing.assert_allclose(df, (xc.spin_interp(z + 1e-6)[0] - xc.spin_interp(z - 1e-6)[0]) / 2e-6, rtol=1e-7)


def test_pw92_spin_fits_have_the_exact_high_density_logarithms():
    """As rs -> 0 the G form tends to A ln rs + const.  The exact RPA
    coefficients: (1 - ln 2) / pi^2 unpolarised, half of it fully
    polarised, and 1 / (6 pi^2) for the spin stiffness -alpha_c."""
    c0 = (1.0 - np.log(2.0)) / np.pi ** 2
    assert abs(xc.PW92_A - c0) / c0 < 1e-4
    assert abs(xc.PW92_POL[0] - c0 / 2) / (c0 / 2) < 1e-4
    assert abs(xc.PW92_MALPHA[0] - 1.0 / (6 * np.pi ** 2)) * 6 * np.pi ** 2 < 1e-4
    rs = np.array([1e-8, 1e-9])
    for A, a1, beta in (xc.PW92_POL, xc.PW92_MALPHA):
        G, _ = xc.pw92_G(rs, A, a1, beta)
        assert abs((G[0] - G[1]) / np.log(rs[0] / rs[1]) - A) < 1e-6


def test_pw92_spin_fits_have_no_sqrt_rs_term():
    """The fully polarised fit and the spin stiffness fit obey the same
    exact high-density form as the unpolarised one (A ln r_s + const +
    O(r_s ln r_s), no r_s^(1/2) term), which fixes b2 = 2 A b1^2 in each."""
    from test_oracle_pins import sqrt_rs_coefficient
    for A, a1, beta in (xc.PW92_POL, xc.PW92_MALPHA):
        b1, b2 = beta[0], beta[1]
        assert abs(b2 - 2.0 * A * b1 * b1) / b2 < 1e-4
        coef = sqrt_rs_coefficient(lambda r: xc.pw92_G(np.array([r]), A, a1, beta)[0][0], A)
        assert abs(coef) < 2e-4 * (2.0 * A * 2.0 * A * b1), (A, coef)


def test_spin_occupations_common_fermi_level():
    rng = np.random.default_rng(4)
    lu = np.sort(rng.uniform(-1, 1, 10))
    ld = np.sort(rng.uniform(-1, 1, 10))
    mu, fu, fd = scf.occupations_spin(lu, ld, 9.0, 0.01)
    assert abs(fu.sum() + fd.sum() - 9.0) < 1e-12
    np.testing.assert_allclose(fu, scf.fermi(lu, mu, 0.01), rtol=0, atol=0)
    # equal spectra: half the unpolarised occupations at the same mu
    mu2, g = scf.occupations(lu, 9.0, 0.01)
    mu3, f3u, f3d = scf.occupations_spin(lu, lu, 9.0, 0.01)
    assert abs(mu2 - mu3) < 1e-12
    np.testing.assert_allclose(f3u, 0.5 * g, atol=1e-14)
    np.testing.assert_allclose(f3d, 0.5 * g, atol=1e-14)


def test_spin_preconditioner_filters_the_total_and_keeps_the_moment():
    s = W.tiny_system(n=(14, 14, 16))
    rng = np.random.default_rng(5)
    fu, fd = rng.standard_normal(s.nd), rng.standard_normal(s.nd)
    out = scf.spin_precondition(s, np.concatenate([fu, fd]), 1.0)
    np.testing.assert_allclose(out[:s.nd] + out[s.nd:], scf.kerker(s, fu + fd, 1.0), atol=1e-13)
    np.testing.assert_allclose(out[:s.nd] - out[s.nd:], fu - fd, atol=1e-13)
    same = scf.spin_precondition(s, np.concatenate([fu, fu]), 1.0)
    np.testing.assert_allclose(same[:s.nd], scf.kerker(s, fu, 1.0), atol=1e-13)


def test_spin_scf_with_symmetric_start_is_the_unpolarised_scf():
    """Equal spin densities and equal starting blocks stay symmetric; the
    spin SCF then reproduces the pinned unpolarised SCF step for step (free
    energy, residual, eigenvalues), which pins its occupations, energy
    terms, mixing and schedule."""
    s = W.config1(0)
    sp = replace(s, spin=2, spin_zeta0=0.0)
    X0 = W.initial_orbitals(s.nd, s.n_states, s.seed)
    r1 = scf.scf(s, X0, max_iter=3, tol=0.0)
    r2 = scf.scf_spin(sp, X0, X0, max_iter=3, tol=0.0)
    for a, b in zip(r1.history, r2.history):
        assert abs(a["free"] - b["free"]) <= 1e-11
        assert abs(a["residual"] - b["residual"]) <= 1e-11
        np.testing.assert_allclose(b["lam"][0], a["lam"], atol=1e-11)
        np.testing.assert_allclose(b["lam"][1], a["lam"], atol=1e-11)
        assert abs(b["magnetization"]) < 1e-12


def test_spin_golden_is_current_and_a_fixed_point():
    import json
    import os
    ref = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cfg1s_spin_scf.json")))
    s = W.config1_spin(0)
    Xu, Xd = W.initial_orbitals_spin(s.nd, s.n_states, s.seed)
    r = scf.scf_spin(s, Xu, Xd, max_iter=2, tol=0.0)
    for k in range(2):
        assert abs(r.history[k]["free"] / s.n_atoms - ref["trajectory"][k]["free_per_atom"]) <= 1e-12
        assert abs(r.history[k]["residual"] - ref["trajectory"][k]["residual"]) <= 1e-12
    fu, fd = np.array(ref["occ_up"]), np.array(ref["occ_dn"])
    assert abs(fu.sum() + fd.sum() - s.n_electrons) <= 1e-12
    np.testing.assert_allclose(fu, scf.fermi(np.array(ref["eig_up"]), ref["mu"], s.kT), atol=1e-12)
    np.testing.assert_allclose(fd, scf.fermi(np.array(ref["eig_dn"]), ref["mu"], s.kT), atol=1e-12)
    # the moment is the occupation imbalance
    assert abs(ref["magnetization"] - (fu.sum() - fd.sum())) <= 1e-8
    assert 0.9 < abs(ref["magnetization"]) <= 1.0
    assert ref["residual"] < ref["tol"]
