"""Writes the stored SCF reference values under tests/golden/ from the CPU
oracle alone (no GPU code is imported).

    python tests/golden/make_golden.py [file names to rewrite; default all]

cfg1_scf.json: the 8-atom, 24^3 system (seed 0) iterated by the oracle's
SCF (Sec. 2.1: Chebyshev-filtered subspace iteration with linear density
mixing) from the seeded random block until the density residual is below
1e-10: the free energy per atom and eigenvalues at the fixed point, the
per-iteration trajectory of the first iterations, and the density at seeded
sample points together with its integrals.

cfg1_scf_pulay.json: the same system and record with the restarted periodic
Pulay mixing of Sec. 2.1 (history 7, period 2) in place of linear mixing.

cfg1s_spin_scf.json: the spin-polarised config 1 (workloads.config1_spin(0),
15 electrons) iterated by the oracle's spin SCF from the seeded (up, down)
blocks to a residual below 1e-10: free energy, both spectra, occupations,
the moment, the trajectory of the first iterations and samples of both
output spin densities.
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import scf  # noqa: E402

N_TRAJ = 12
N_SAMPLES = 64


def cfg1_scf(pulay=None):
    s = W.config1(0)
    if pulay is not None:
        s.pulay_history, s.pulay_period, s.pulay_restart = pulay
    X0 = W.initial_orbitals(s.nd, s.n_states, s.seed)
    r = scf.scf(s, X0, max_iter=200, tol=1e-10)
    dv = float(np.prod(s.h))
    idx = np.sort(np.random.default_rng(2024).choice(s.nd, N_SAMPLES, replace=False))
    last = r.history[-1]
    return {
        "system": "workloads.config1(0)" + ("" if pulay is None else
                                            " with pulay_history, pulay_period, pulay_restart = %d, %d, %d" % pulay),
        "tol": 1e-10,
        "n_iter": len(r.history),
        "free_per_atom": last["free"] / s.n_atoms,
        "terms": {k: last[k] for k in ("band", "exc", "vxc_dc", "elec", "self", "corr", "entropy", "free")},
        "mu": float(r.mu),
        "eig": [float(x) for x in r.lam],
        "occ": [float(x) for x in r.g],
        "residual": last["residual"],
        "trajectory": [{"free_per_atom": h["free"] / s.n_atoms, "residual": h["residual"],
                        "eig_min": float(h["lam"][0]), "eig_max": float(h["lam"][-1])}
                       for h in r.history[:N_TRAJ]],
        "rho_out_samples": {"index": [int(i) for i in idx], "value": [float(r.rho_out[i]) for i in idx]},
        "rho_out_integrals": {"int_rho": float(dv * r.rho_out.sum()), "int_rho2": float(dv * (r.rho_out ** 2).sum())},
    }


def cfg1s_spin_scf():
    s = W.config1_spin(0)
    Xu, Xd = W.initial_orbitals_spin(s.nd, s.n_states, s.seed)
    r = scf.scf_spin(s, Xu, Xd, max_iter=300, tol=1e-10)
    nd = s.nd
    idx = np.sort(np.random.default_rng(2025).choice(nd, N_SAMPLES, replace=False))
    last = r.history[-1]
    return {
        "system": "workloads.config1_spin(0)",
        "tol": 1e-10,
        "n_iter": len(r.history),
        "free_per_atom": last["free"] / s.n_atoms,
        "terms": {k: last[k] for k in ("band", "exc", "vxc_dc", "elec", "self", "corr", "entropy", "free")},
        "mu": float(r.mu),
        "magnetization": last["magnetization"],
        "eig_up": [float(x) for x in r.lam[0]],
        "eig_dn": [float(x) for x in r.lam[1]],
        "occ_up": [float(x) for x in r.f[0]],
        "occ_dn": [float(x) for x in r.f[1]],
        "residual": last["residual"],
        "trajectory": [{"free_per_atom": h["free"] / s.n_atoms, "residual": h["residual"],
                        "magnetization": h["magnetization"]} for h in r.history[:N_TRAJ]],
        "rho_out_samples": {"index": [int(i) for i in idx],
                            "up": [float(r.rho_out[i]) for i in idx],
                            "dn": [float(r.rho_out[nd + i]) for i in idx]},
    }


def main():
    jobs = (("cfg1_scf.json", lambda: cfg1_scf()), ("cfg1_scf_pulay.json", lambda: cfg1_scf((7, 2, 1))),
            ("cfg1s_spin_scf.json", cfg1s_spin_scf))
    for name, job in jobs:
        if len(sys.argv) > 1 and name not in sys.argv[1:]:
            continue
        out = os.path.join(HERE, name)
        with open(out, "w") as f:
            json.dump(job(), f, indent=1)
        print("wrote", out)


if __name__ == "__main__":
    main()
