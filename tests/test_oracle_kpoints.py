"""Pins of the oracle's Bloch k-point form against facts it does not compute
itself: the closed-form free-electron spectrum, the Gamma-point Hamiltonian
at k = 0, Hermiticity, time reversal, band folding of a supercell (which
fixes every phase, projectors included), and the k = 0 SCF against the real
Gamma-point SCF."""
from dataclasses import replace

import numpy as np

import workloads as W
from oracle import atoms, fd, hamiltonian, kpoints, scf


def _tiny():
    return W.tiny_system(n=(8, 7, 9), L=(2.6, 2.4, 2.9), n_atoms=1, seed=3)


def _veff(s, seed=0):
    return np.random.default_rng(seed).uniform(-1, 1, s.nd)


def test_bloch_hamiltonian_is_hermitian_and_reduces_to_gamma():
    s = _tiny()
    v = _veff(s)
    k = np.array([0.7, -0.4, 0.3])
    H = kpoints.dense_H_k(s, v, kpoints.projectors_k(s, k), k)
    assert np.max(np.abs(H - H.conj().T)) < 1e-13
    H0 = kpoints.dense_H_k(s, v, kpoints.projectors_k(s, [0, 0, 0]), [0, 0, 0])
    assert np.max(np.abs(H0 - hamiltonian.dense_H(s, v, atoms.projectors(s)))) < 1e-12
    em = np.linalg.eigvalsh(kpoints.dense_H_k(s, v, kpoints.projectors_k(s, -k), -k))
    assert np.max(np.abs(np.linalg.eigvalsh(H) - em)) < 1e-12


def test_free_electron_bloch_spectrum_is_the_stencil_symbol_at_shifted_wavenumbers():
    s = replace(_tiny(), nl_lmax=-1, gamma=None)
    k = np.array([0.7, -0.4, 0.3])
    ev = np.sort(np.linalg.eigvalsh(kpoints.dense_H_k(s, np.zeros(s.nd), [], k)))
    cf = []
    for mx in range(s.n[0]):
        for my in range(s.n[1]):
            for mz in range(s.n[2]):
                cf.append(sum(-0.5 * fd.symbol((2 * np.pi * m / s.L[d] + k[d]) * s.h[d], s.fd_half_order) / s.h[d] ** 2
                              for d, m in enumerate((mx, my, mz))))
    assert np.max(np.abs(ev - np.sort(cf))) < 1e-11


def test_supercell_gamma_spectrum_folds_onto_two_k_points():
    """The Gamma-point Hamiltonian of the 2x1x1 supercell (atoms and V_eff
    repeated) has the union of the primitive cell's spectra at k = 0 and
    k = pi / L_x."""
    s = _tiny()
    v = _veff(s, 1)
    nx, ny, nz = s.n
    sc = replace(s, n=(2 * nx, ny, nz), L=(2 * s.L[0], s.L[1], s.L[2]),
                 pos=np.vstack([s.pos, s.pos + [s.L[0], 0, 0]]), Z=np.tile(s.Z, 2), rc_loc=np.tile(s.rc_loc, 2),
                 gamma=np.tile(s.gamma, (2, 1)), n_electrons=2 * s.n_electrons)
    vsc = np.tile(v.reshape(nz, ny, nx), (1, 1, 2)).reshape(-1)
    e_sc = np.sort(np.linalg.eigvalsh(hamiltonian.dense_H(sc, vsc, atoms.projectors(sc))))
    ka = np.array([np.pi / s.L[0], 0.0, 0.0])
    e_fold = np.sort(np.concatenate([
        np.linalg.eigvalsh(kpoints.dense_H_k(s, v, kpoints.projectors_k(s, [0, 0, 0]), [0, 0, 0])),
        np.linalg.eigvalsh(kpoints.dense_H_k(s, v, kpoints.projectors_k(s, ka), ka))]))
    assert np.max(np.abs(e_sc - e_fold)) < 1e-11


def test_rayleigh_ritz_k_recovers_exact_eigenpairs_and_bounds_hold():
    s = _tiny()
    v = _veff(s, 2)
    k = np.array([0.3, 0.5, -0.6])
    pk = kpoints.projectors_k(s, k)
    H = kpoints.dense_H_k(s, v, pk, k)
    lam, V = np.linalg.eigh(H)
    lo, hi = kpoints.spectrum_bounds_k(s, v, pk)
    assert lo <= lam[0] + 1e-12 and lam[-1] <= hi + 1e-12
    # a random mixture of the lowest 5 eigenvectors spans them exactly
    rng = np.random.default_rng(3)
    C = rng.standard_normal((5, 5)) + 1j * rng.standard_normal((5, 5))
    Y = C @ V[:, :5].T
    X, ritz = kpoints.rayleigh_ritz_k(s, v, pk, Y, k)
    np.testing.assert_allclose(ritz, lam[:5], atol=1e-11)
    np.testing.assert_allclose(s.dV * (np.conj(X) @ X.T), np.eye(5), atol=1e-11)


def test_k_occupations_single_point_is_gamma_and_weights_count_electrons():
    rng = np.random.default_rng(4)
    l1, l2 = np.sort(rng.uniform(-1, 1, 8)), np.sort(rng.uniform(-1, 1, 8))
    mu_g, g = scf.occupations(l1, 7.0, 0.01)
    mu_k, gs = kpoints.occupations_k([l1], [1.0], 7.0, 0.01)
    assert abs(mu_g - mu_k) < 1e-12 and np.max(np.abs(gs[0] - g)) < 1e-12
    mu2, gs2 = kpoints.occupations_k([l1, l2], [0.25, 0.75], 7.0, 0.01)
    assert abs(0.25 * gs2[0].sum() + 0.75 * gs2[1].sum() - 7.0) < 1e-12


def test_k0_scf_equals_the_gamma_scf():
    s = W.config1(0)
    X0 = W.initial_orbitals(s.nd, s.n_states, s.seed)
    r1 = scf.scf(s, X0, max_iter=3, tol=0.0)
    r2 = kpoints.scf_k(s, np.zeros((1, 3)), np.ones(1), [X0], max_iter=3, tol=0.0)
    for a, b in zip(r1.history, r2["history"]):
        assert abs(a["free"] - b["free"]) < 1e-10
        assert abs(a["residual"] - b["residual"]) < 1e-10
        np.testing.assert_allclose(b["lam"][0], a["lam"], atol=1e-10)
