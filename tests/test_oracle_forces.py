"""Pins of the oracle's Hellmann-Feynman forces: each part is the negative
derivative of the energy term it comes from (central differences of the
oracle's energy routines, which the force code does not call), and the total
is the derivative of the self-consistent free energy (the Hellmann-Feynman
theorem)."""
from dataclasses import replace

import numpy as np

import workloads as W
from oracle import atoms, electrostatics, forces, scf


def _moved(s, I, a, step):
    pos = s.pos.copy()
    pos[I, a] += step
    return replace(s, pos=pos)


def _system():
    # projector cutoff at 6 rc: the truncated Gaussian tail (e^-36) is below
    # rounding, so no support point crossing the sphere changes the energy
    return replace(W.tiny_system(n=(14, 16, 18)), rcut_nl=6.0, n_states=8)


def test_overlap_force_is_minus_the_gradient_of_the_overlap_energy():
    s = W.tiny_system(n=(14, 16, 18), n_atoms=3, seed=8)
    F = forces.overlap_forces(s)
    h = 1e-5
    for I in range(s.n_atoms):
        for a in range(3):
            fd = -(atoms.overlap_correction(_moved(s, I, a, h)) - atoms.overlap_correction(_moved(s, I, a, -h))) / (2 * h)
            assert abs(fd - F[I, a]) <= 1e-8 * max(1.0, abs(fd)), (I, a, fd, F[I, a])
    # Newton's third law over all pairs and images
    assert np.max(np.abs(F.sum(axis=0))) < 1e-12


def test_local_force_is_minus_the_gradient_of_the_electrostatic_energy_at_fixed_density():
    """E_loc(R) = 1/2 dV sum (rho + b_R) phi_R - E_self(R) with rho held fixed."""
    s = _system()
    rho = np.random.default_rng(6).uniform(0.1, 1.0, s.nd)

    def E(sx):
        b = atoms.pseudocharge(sx)
        phi = electrostatics.hartree_ionic_potential(sx, rho, b)
        return 0.5 * sx.dV * float(np.sum((rho + b) * phi)) - atoms.self_energy(sx)
    b = atoms.pseudocharge(s)
    F = forces.local_forces(s, electrostatics.hartree_ionic_potential(s, rho, b))
    h = 1e-4
    for I in range(s.n_atoms):
        for a in range(3):
            fd = -(E(_moved(s, I, a, h)) - E(_moved(s, I, a, -h))) / (2 * h)
            assert abs(fd - F[I, a]) <= 1e-7 * max(1.0, abs(fd)), (I, a, fd, F[I, a])


def test_nonlocal_force_is_minus_the_gradient_of_the_projector_energy_at_fixed_orbitals():
    """E_nl(R) = sum_n w_n sum_{I,k} gamma_Ik (dV chi_Ik^T psi_n)^2 with the
    projector tables of atoms.projectors and fixed orbitals."""
    s = _system()
    rng = np.random.default_rng(7)
    X = rng.standard_normal((5, s.nd))
    w = rng.uniform(0.0, 2.0, 5)

    def E(sx):
        e = 0.0
        for p in atoms.projectors(sx):
            P = sx.dV * (X[:, p.idx] @ p.chi.T)       # (n, 4)
            e += float(np.sum(w[:, None] * p.gamma[None, :] * P * P))
        return e
    F = forces.nonlocal_forces(s, [X], [w])
    h = 1e-4
    for I in range(s.n_atoms):
        for a in range(3):
            fd = -(E(_moved(s, I, a, h)) - E(_moved(s, I, a, -h))) / (2 * h)
            assert abs(fd - F[I, a]) <= 1e-7 * max(1.0, abs(fd)), (I, a, fd, F[I, a])


def test_forces_are_the_derivative_of_the_self_consistent_free_energy():
    """Hellmann-Feynman: at self-consistency (residual 1e-12) the force equals
    minus the derivative of the converged free energy (central differences,
    step 1e-3 Bohr)."""
    s = _system()
    X0 = W.initial_orbitals(s.nd, s.n_states, 3)

    def run(sx):
        return scf.scf(sx, X0, max_iter=400, tol=1e-12, degree=16)
    r = run(s)
    st = scf.setup(s)
    phi, _, _, _ = scf.potential(s, st, r.rho_in)
    F = forces.forces(s, phi, [r.X], [r.g])
    for I, a in ((0, 0), (1, 2)):
        Ep = run(_moved(s, I, a, 1e-3)).history[-1]["free"]
        Em = run(_moved(s, I, a, -1e-3)).history[-1]["free"]
        fd = -(Ep - Em) / 2e-3
        assert abs(fd - F[I, a]) <= 1e-7, (I, a, fd, F[I, a])
    # two atoms: the forces are nearly opposite (the grid breaks translation
    # invariance only slightly)
    assert np.max(np.abs(F.sum(axis=0))) < 1e-5
