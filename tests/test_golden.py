"""The stored SCF reference (tests/golden/cfg1_scf.json) is what the oracle
computes now: its first iterations are recomputed and compared, and the
stored fixed point satisfies the constraints that hold at any SCF fixed
point (electron count, occupations from the Fermi function at mu)."""
import json
import os

import numpy as np

import workloads as W
from oracle import scf

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cfg1_scf.json")


def test_golden_trajectory_is_current():
    ref = json.load(open(GOLDEN))
    s = W.config1(0)
    X0 = W.initial_orbitals(s.nd, s.n_states, s.seed)
    r = scf.scf(s, X0, max_iter=3, tol=0.0)
    for k in range(3):
        assert abs(r.history[k]["free"] / s.n_atoms - ref["trajectory"][k]["free_per_atom"]) <= 1e-12
        assert abs(r.history[k]["residual"] - ref["trajectory"][k]["residual"]) <= 1e-12


def test_golden_fixed_point_constraints():
    ref = json.load(open(GOLDEN))
    s = W.config1(0)
    lam, occ, mu = np.array(ref["eig"]), np.array(ref["occ"]), ref["mu"]
    assert np.all(np.diff(lam) >= 0)
    assert abs(occ.sum() - s.n_electrons) <= 1e-12
    assert np.allclose(occ, 2.0 / (1.0 + np.exp((lam - mu) / s.kT)), atol=1e-12, rtol=0)
    assert abs(ref["rho_out_integrals"]["int_rho"] - s.n_electrons) <= 1e-9
    assert ref["residual"] < ref["tol"]


GOLDEN_PULAY = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cfg1_scf_pulay.json")


def test_pulay_golden_trajectory_is_current():
    """First iterations of the stored Pulay run (Pulay steps at iterations 1
    and 3 with period 2) are what the oracle computes now."""
    ref = json.load(open(GOLDEN_PULAY))
    s = W.config1(0)
    s.pulay_history, s.pulay_period, s.pulay_restart = 7, 2, 1
    X0 = W.initial_orbitals(s.nd, s.n_states, s.seed)
    r = scf.scf(s, X0, max_iter=5, tol=0.0)
    for k in range(5):
        assert abs(r.history[k]["free"] / s.n_atoms - ref["trajectory"][k]["free_per_atom"]) <= 1e-12
        assert abs(r.history[k]["residual"] - ref["trajectory"][k]["residual"]) <= 1e-12


def test_pulay_and_linear_mixing_reach_the_same_fixed_point():
    """The mixing scheme changes the path, not the fixed point: the Pulay run
    converges in fewer iterations to the free energy, occupied eigenvalues
    and density of the linear-mixing run (to the 1e-10 residual both stop
    at)."""
    lin, pul = json.load(open(GOLDEN)), json.load(open(GOLDEN_PULAY))
    assert pul["n_iter"] < lin["n_iter"]
    assert abs(pul["free_per_atom"] - lin["free_per_atom"]) <= 1e-10
    occ = np.array(lin["occ"]) > 1e-4
    assert np.max(np.abs(np.array(pul["eig"])[occ] - np.array(lin["eig"])[occ])) <= 1e-9
    assert pul["rho_out_samples"]["index"] == lin["rho_out_samples"]["index"]
    assert np.max(np.abs(np.array(pul["rho_out_samples"]["value"]) - np.array(lin["rho_out_samples"]["value"]))) <= 1e-9
