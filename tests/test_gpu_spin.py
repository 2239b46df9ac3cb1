"""GPU parity of the spin-polarised form (eq. (1)-(2) with a spin index;
Sec. 2.1 for mixing both spin densities as one vector) against the oracle:
the LSDA potential, common-mu occupations, the spin mixing step, a
spin-symmetric SCF against the unpolarised SCF, and the converged spin SCF
of the 15-electron config-1 variant against the stored oracle run."""
import json
import os
from dataclasses import replace

import numpy as np
import pytest

import workloads as W
from oracle import atoms, scf

from gpu_helpers import log, rel_err, require_gpu, to_np

pytestmark = pytest.mark.gpu


def _spin_densities(s, seed):
    """SAD density split with a smooth, seeded polarisation field; one region
    fully polarised down to the floor."""
    rng = np.random.default_rng(seed)
    rho = atoms.sad_density(s)
    z = np.clip(0.6 * np.sin(np.arange(s.nd) * 2 * np.pi / s.n[0] + rng.uniform(0, 6)), -1, 1)
    up, dn = 0.5 * (1 + z) * rho, 0.5 * (1 - z) * rho
    dn[: s.nd // 50] = 0.0
    return up, dn


def test_potential_spin_matches_oracle():
    torch = require_gpu()
    from paper_2005_10431_amd import Context
    s = W.config1_spin(0)
    ctx = Context(s)
    try:
        st = scf.setup(s)
        up, dn = _spin_densities(s, 1)
        phi, exc, vu, vd, veu, ved = scf.potential_spin(s, st, up, dn)
        z = lambda n: torch.zeros(n, dtype=torch.float64, device="cuda")
        P, E, V, VE = z(s.nd), z(s.nd), z(2 * s.nd), z(2 * s.nd)
        ctx.potential_spin(torch.from_numpy(np.concatenate([up, dn])).cuda(), P, E, V, VE)
        V, VE = to_np(V), to_np(VE)
        assert np.max(np.abs(to_np(P) - phi)) <= 1e-11 * max(1.0, np.max(np.abs(phi)))
        assert rel_err(to_np(E), exc) <= 1e-13
        assert rel_err(V[:s.nd], vu) <= 1e-13 and rel_err(V[s.nd:], vd) <= 1e-13
        assert np.max(np.abs(VE[:s.nd] - veu)) <= 1e-11 * max(1.0, np.max(np.abs(veu)))
        assert np.max(np.abs(VE[s.nd:] - ved)) <= 1e-11 * max(1.0, np.max(np.abs(ved)))
    finally:
        ctx.close()


@pytest.mark.parametrize("zeta0", [1.0 / 15.0, -0.4, 1.0])
def test_sad_density_spin_matches_oracle(zeta0):
    """The split atomic-density guess is formed in the library (spin up
    (1 + zeta0) rho / 2, down (1 - zeta0) rho / 2); zeta0 outside [-1, 1]
    is rejected."""
    torch = require_gpu()
    from paper_2005_10431_amd import Context, SparcError
    s = replace(W.config1_spin(0), spin_zeta0=zeta0)
    ctx = Context(s)
    try:
        up, dn = scf.sad_density_spin(s)
        rho = torch.full((2 * s.nd,), 7.0, dtype=torch.float64, device="cuda")
        ctx.sad_density_spin(zeta0, rho)
        r = to_np(rho)
        assert np.max(np.abs(r[:s.nd] - up)) <= 1e-13 * np.max(up)
        assert np.max(np.abs(r[s.nd:] - dn)) <= 1e-13 * max(np.max(up), 1e-300)
        assert abs(s.dV * r.sum() - s.n_electrons) <= 1e-11 * s.n_electrons
        for bad in (1.5, -1.01, float("nan")):
            with pytest.raises(SparcError):
                ctx.sad_density_spin(bad, rho)
    finally:
        ctx.close()


def test_occupations_spin_match_oracle():
    torch = require_gpu()
    from paper_2005_10431_amd import Context
    s = W.config1_spin(0)
    ctx = Context(s)
    try:
        rng = np.random.default_rng(2)
        lu = np.sort(rng.uniform(-0.5, 0.3, s.n_states))
        ld = np.sort(rng.uniform(-0.5, 0.3, s.n_states))
        mu_r, fu, fd = scf.occupations_spin(lu, ld, s.n_electrons, s.kT)
        occ = torch.zeros(2 * s.n_states, dtype=torch.float64, device="cuda")
        mu = torch.zeros(1, dtype=torch.float64, device="cuda")
        ctx.occupations_spin(torch.from_numpy(np.concatenate([lu, ld])).cuda(), occ, mu)
        o = to_np(occ)
        assert abs(float(mu.item()) - mu_r) <= 1e-12
        np.testing.assert_allclose(o, np.concatenate([fu, fd]), rtol=0, atol=1e-12)
        assert abs(o.sum() - s.n_electrons) <= 1e-12
    finally:
        ctx.close()


@pytest.mark.parametrize("m,period,restart,q0", [(0, 1, 0, 0.0), (0, 1, 0, 1.0), (4, 2, 1, 1.0), (4, 1, 0, 0.0)])
def test_mix_spin_matches_oracle(m, period, restart, q0):
    """Both spins mixed as one vector; the preconditioner acts on the total.
    Same inputs per iteration on both sides (the oracle's trajectory on a
    moment-conserving contraction); bars as in the one-spin mixer test."""
    torch = require_gpu()
    from paper_2005_10431_amd import Context
    s = W.tiny_system(n=(14, 16, 18))
    nd = s.nd
    log(f"spin mix parity m={m} period={period} restart={restart} q0={q0}")
    rng = np.random.default_rng(40 + m)
    c0 = rng.uniform(-0.5, 0.5, 2 * nd)
    c0[:nd] -= c0[:nd].mean()
    c0[nd:] -= c0[nd:].mean()

    def g(x):
        out = np.empty_like(x)
        for k in (0, 1):
            v = x[k * nd:(k + 1) * nd]
            mu = v.mean()
            out[k * nd:(k + 1) * nd] = mu + c0[k * nd:(k + 1) * nd] + 0.85 * (
                0.5 * (np.roll(v, 1) + np.roll(v, -5)) - mu)
        return out
    x = rng.uniform(0.5, 1.5, 2 * nd)
    mixer = scf.PeriodicPulay(m, period, 0.3, restart=bool(restart),
                              precondition=lambda f: scf.spin_precondition(s, f, q0))
    ctx = Context(s)
    eps = np.finfo(np.float64).eps
    try:
        hist = torch.empty((2 * m + 2) * 2 * nd, dtype=torch.float64, device="cuda") if m > 0 else None
        rin = torch.empty(2 * nd, dtype=torch.float64, device="cuda")
        rout = torch.empty(2 * nd, dtype=torch.float64, device="cuda")
        for k in range(10):
            ro = g(x)
            rin.copy_(torch.from_numpy(x))
            rout.copy_(torch.from_numpy(ro))
            ctx.mix(rin, rout, 0.3, q0, m, period, restart, hist, k, n_spin=2)
            ref = mixer.step(x, ro - x)
            bar = 1e-13 * np.max(np.abs(ref))
            if mixer.last is not None:
                F, Xd, gamma = mixer.last
                bar += 100 * eps * np.linalg.cond(F.T @ F) * float(
                    np.sum(np.abs(gamma) * np.max(np.abs(Xd), axis=0)))
            err = float(np.max(np.abs(to_np(rin) - ref)))
            assert err <= bar, (k, err, bar)
            x = ref
    finally:
        ctx.close()


def test_spin_scf_with_symmetric_start_matches_unpolarised_scf():
    """Through the C ABI: equal spin densities and equal starting blocks give
    the unpolarised SCF's energies, residuals and eigenvalues."""
    require_gpu()
    from paper_2005_10431_amd.driver import run_scf, run_scf_spin
    s = W.config1(0)
    sp = replace(s, spin=2, spin_zeta0=0.0)
    X0 = W.initial_orbitals(s.nd, s.n_states, s.seed)
    r1 = run_scf(s, X0, max_iter=4, tol=0.0)
    r2 = run_scf_spin(sp, (X0, X0), max_iter=4, tol=0.0)
    for a, b in zip(r1["history"], r2["history"]):
        assert abs(a["free_energy"] - b["free_energy"]) <= 1e-10
        assert abs(a["residual"] - b["residual"]) <= 1e-10
        np.testing.assert_allclose(b["eig_up"], a["eig"], atol=1e-10)
        np.testing.assert_allclose(b["eig_dn"], a["eig"], atol=1e-10)
        assert abs(b["magnetization"]) <= 1e-10
    r1["ctx"].close()
    r2["ctx"].close()


def test_spin_scf_cfg1s_matches_oracle():
    """15-electron config-1 variant, FP64, to a residual of 1e-10 from the
    seeded blocks: same fixed point (free energy, occupied eigenvalues of
    both spins, moment, density samples), iteration count within 2 and the
    first iterations on the oracle's trajectory."""
    require_gpu()
    from paper_2005_10431_amd.driver import run_scf_spin
    ref = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cfg1s_spin_scf.json")))
    s = W.config1_spin(0)
    out = run_scf_spin(s, max_iter=300, tol=ref["tol"])
    h = out["history"]
    F = h[-1]["free_energy"] / s.n_atoms
    occ_u, occ_d = np.array(ref["occ_up"]) > 1e-4, np.array(ref["occ_dn"]) > 1e-4
    dlu = float(np.max(np.abs(h[-1]["eig_up"][occ_u] - np.array(ref["eig_up"])[occ_u])))
    dld = float(np.max(np.abs(h[-1]["eig_dn"][occ_d] - np.array(ref["eig_dn"])[occ_d])))
    log(f"cfg1s spin: {len(h)} iterations (oracle {ref['n_iter']}), dF/atom {abs(F - ref['free_per_atom']):.2e}, "
        f"dlam {max(dlu, dld):.2e}, M {h[-1]['magnetization']:.10f} (oracle {ref['magnetization']:.10f})")
    assert h[-1]["residual"] < ref["tol"]
    assert abs(F - ref["free_per_atom"]) <= 1e-9
    assert max(dlu, dld) <= 1e-8
    assert abs(h[-1]["magnetization"] - ref["magnetization"]) <= 1e-8
    assert abs(len(h) - ref["n_iter"]) <= 2
    for k, r in enumerate(ref["trajectory"]):
        assert abs(h[k]["free_energy"] / s.n_atoms - r["free_per_atom"]) <= 1e-8, k
        assert abs(h[k]["residual"] - r["residual"]) <= 1e-8 * max(1.0, r["residual"]), k
        assert abs(h[k]["magnetization"] - r["magnetization"]) <= 1e-7, k
    rho = to_np(out["rho_out"])
    idx = np.array(ref["rho_out_samples"]["index"])
    for part, off in (("up", 0), ("dn", s.nd)):
        val = np.array(ref["rho_out_samples"][part])
        assert np.max(np.abs(rho[off + idx] - val)) <= 1e-8 * np.max(np.abs(val)), part
    out["ctx"].close()


def test_spin_state_rejects_overlapping_blocks():
    torch = require_gpu()
    from paper_2005_10431_amd import Context, SparcError, make_spin_state
    s = W.config1_spin(0)
    ctx = Context(s)
    try:
        X = torch.zeros((s.n_states + 1, s.nd), dtype=torch.float64, device="cuda")
        rho = torch.ones(2 * s.nd, dtype=torch.float64, device="cuda")
        eig = torch.zeros(2 * s.n_states, dtype=torch.float64, device="cuda")
        occ = torch.zeros_like(eig)
        st = make_spin_state(rho, X[:s.n_states], X[1:], eig, occ, 12)
        with pytest.raises(SparcError) as e:
            ctx.scf_step_spin(st)
        assert e.value.status == 1
    finally:
        ctx.close()


def test_spin_scf_fp32_blocks_reach_the_fp64_fixed_point():
    """The FP32 form of the spin SCF (FP32 blocks, FP64 potential,
    occupations, density and mixing) converged to a residual of 1e-6 lands
    within the FP32 form's target (1e-5 Ha/atom) of the stored FP64 oracle
    fixed point, with the same moment to 1e-4."""
    require_gpu()
    from paper_2005_10431_amd.driver import run_scf_spin
    ref = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cfg1s_spin_scf.json")))
    s = W.config1_spin(0)
    out = run_scf_spin(s, prec="fp32", max_iter=300, tol=1e-6)
    h = out["history"]
    dF = abs(h[-1]["free_energy"] / s.n_atoms - ref["free_per_atom"])
    log(f"cfg1s spin FP32: {len(h)} iterations, dF/atom {dF:.2e}, M {h[-1]['magnetization']:.6f}")
    assert h[-1]["residual"] < 1e-6
    assert dF <= 1e-5
    assert abs(h[-1]["magnetization"] - ref["magnetization"]) <= 1e-4
    out["ctx"].close()


def test_spin_scf_with_pulay_matches_oracle():
    """cfg1s with restarted periodic Pulay mixing over the doubled vector
    (history 7, period 2): trajectory, fixed point and moment against the
    oracle's spin SCF with the same mixing."""
    require_gpu()
    from paper_2005_10431_amd.driver import run_scf_spin
    s = replace(W.config1_spin(0), pulay_history=7, pulay_period=2, pulay_restart=1)
    Xu, Xd = W.initial_orbitals_spin(s.nd, s.n_states, s.seed)
    r = scf.scf_spin(s, Xu, Xd, max_iter=300, tol=1e-10)
    out = run_scf_spin(s, (Xu, Xd), max_iter=300, tol=1e-10)
    h = out["history"]
    log(f"cfg1s Pulay: {len(h)} iterations (oracle {len(r.history)}), M {h[-1]['magnetization']:.8f}")
    for k in range(min(10, len(r.history))):
        assert abs(h[k]["free_energy"] - r.history[k]["free"]) <= 1e-8, k
    assert h[-1]["residual"] < 1e-10
    assert abs(h[-1]["free_energy"] - r.history[-1]["free"]) <= 1e-9
    assert abs(h[-1]["magnetization"] - r.history[-1]["magnetization"]) <= 1e-8
    assert abs(len(h) - len(r.history)) <= 2
    out["ctx"].close()
