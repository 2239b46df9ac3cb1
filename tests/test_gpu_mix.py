"""GPU parity of the density mixing step (Sec. 2.1: restarted periodic Pulay
mixing with a real-space preconditioner) against the oracle's mixer, and of a
Pulay-mixed SCF run against the stored oracle run.

Mixer parity: both sides receive the same (rho_in, rho_out) at every
iteration, taken from the oracle's own trajectory on a charge-conserving
linear contraction, so each GPU output is compared with the oracle output of
the same inputs.  Linear steps agree to rounding (1e-13 of max |x|).  A Pulay
step solves the normal equations dF^T dF gamma = dF^T f, whose solution is
perturbed by up to about cond(dF^T dF) * eps relative to |gamma| when the two
sides round differently; the bar adds 100 eps cond |gamma_j| |dX_j| summed
over the columns (computed from the oracle's matrices) to the rounding bar.
"""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import scf

from gpu_helpers import log, require_gpu, to_np

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


def _contraction(nd, seed):
    """A map x -> x_out that keeps sum(x) (like rho_in -> rho_out) and
    contracts the rest with factor 0.85 around a seeded fixed point."""
    rng = np.random.default_rng(seed)
    c0 = rng.uniform(-0.5, 0.5, nd)
    c0 -= c0.mean()

    def g(x):
        mu = x.mean()
        return mu + c0 + 0.85 * (0.5 * (np.roll(x, 1) + np.roll(x, -7)) - mu)
    return g, rng.uniform(0.5, 1.5, nd)


@pytest.mark.parametrize("m,period,restart,q0", [(3, 2, 0, 0.0), (3, 1, 1, 1.0), (10, 1, 0, 1.0), (10, 2, 1, 0.0),
                                                 (0, 1, 0, 1.0), (0, 1, 0, 0.0)])
def test_mix_matches_oracle(m, period, restart, q0):
    torch = require_gpu()
    from paper_2005_10431_amd import Context
    s = W.tiny_system(n=(14, 16, 18))
    nd = s.nd
    log(f"mix parity m={m} period={period} restart={restart} q0={q0} nd={nd}")
    g, x = _contraction(nd, 31 + m)
    mixer = scf.PeriodicPulay(m, period, 0.3, s, q0, bool(restart))
    ctx = Context(s)
    try:
        hist = torch.empty((2 * m + 2) * nd, dtype=torch.float64, device="cuda") if m > 0 else None
        rin = torch.empty(nd, dtype=torch.float64, device="cuda")
        rout = torch.empty(nd, dtype=torch.float64, device="cuda")
        n_pulay = 0
        for k in range(16):
            ro = g(x)
            rin.copy_(torch.from_numpy(x))
            rout.copy_(torch.from_numpy(ro))
            ctx.mix(rin, rout, 0.3, q0, m, period, restart, hist, k)
            ref = mixer.step(x, ro - x)
            got = to_np(rin)
            bar = 1e-13 * np.max(np.abs(ref))
            if mixer.last is not None:
                F, Xd, gamma = mixer.last
                cond = np.linalg.cond(F.T @ F)
                bar += 100 * EPS * cond * float(np.sum(np.abs(gamma) * np.max(np.abs(Xd), axis=0)))
                n_pulay += 1
            err = float(np.max(np.abs(got - ref)))
            assert err <= bar, (k, err, bar)
            x = ref
        expect = 0 if m == 0 else len([k for k in range(1, 16) if (k + 1) % period == 0])
        assert n_pulay == expect
    finally:
        ctx.close()


def test_mix_singular_normal_equations_are_reported():
    """A repeated iterate gives dF = 0: the call reports SPARC_ERR_SINGULAR
    and leaves the linear step (gamma = 0)."""
    torch = require_gpu()
    from paper_2005_10431_amd import Context, SparcError
    s = W.tiny_system(n=(14, 16, 18))
    nd = s.nd
    g, x = _contraction(nd, 5)
    ro = g(x)
    ctx = Context(s)
    try:
        hist = torch.empty(6 * nd, dtype=torch.float64, device="cuda")
        rin = torch.from_numpy(x).cuda()
        rout = torch.from_numpy(ro).cuda()
        ctx.mix(rin, rout, 0.3, 0.0, 2, 1, False, hist, 0)
        rin.copy_(torch.from_numpy(x))
        with pytest.raises(SparcError) as e:
            ctx.mix(rin, rout, 0.3, 0.0, 2, 1, False, hist, 1)
        assert e.value.status == 9
        np.testing.assert_allclose(to_np(rin), x + 0.3 * (ro - x), rtol=0, atol=1e-15 * np.max(np.abs(x)))
    finally:
        ctx.close()


def test_mix_rejects_bad_arguments():
    torch = require_gpu()
    from paper_2005_10431_amd import Context, SparcError
    s = W.tiny_system(n=(14, 16, 18))
    ctx = Context(s)
    try:
        rin = torch.ones(s.nd, dtype=torch.float64, device="cuda")
        rout = torch.ones(s.nd, dtype=torch.float64, device="cuda")
        hist = torch.zeros(24 * s.nd, dtype=torch.float64, device="cuda")
        for args in ((0.3, 0.0, 11, 1, False, hist, 0), (0.3, 0.0, 2, 0, False, hist, 0),
                     (0.3, 0.0, 2, 1, False, None, 0), (0.0, 0.0, 0, 1, False, None, 0),
                     (0.3, -1.0, 0, 1, False, None, 0), (0.3, 0.0, 2, 1, False, hist, -1)):
            with pytest.raises(SparcError) as e:
                ctx.mix(rin, rout, *args)
            assert e.value.status == 1, args
        assert float(rin.min()) == 1.0 and float(rin.max()) == 1.0
    finally:
        ctx.close()


GOLDEN_PULAY = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cfg1_scf_pulay.json")


def test_scf_cfg1_pulay_matches_oracle():
    """The 8-atom 24^3 SCF with restarted periodic Pulay mixing (history 7,
    period 2) against the stored oracle run: same fixed point and iteration
    count, and the first iterations follow the oracle's trajectory."""
    require_gpu()
    from paper_2005_10431_amd.driver import run_scf
    ref = json.load(open(GOLDEN_PULAY))
    s = W.config1(0)
    X0 = W.initial_orbitals(s.nd, s.n_states, s.seed)
    out = run_scf(s, X0, prec="fp64", max_iter=200, tol=ref["tol"], pulay_history=7, pulay_period=2,
                  pulay_restart=True)
    hist = out["history"]
    F = hist[-1]["free_energy"] / s.n_atoms
    lam = to_np(out["eig"])
    dF = abs(F - ref["free_per_atom"])
    occ = np.array(ref["occ"]) > 1e-4
    dlam = float(np.max(np.abs(lam[occ] - np.array(ref["eig"])[occ])))
    dev = max(abs(hist[k]["free_energy"] / s.n_atoms - r["free_per_atom"]) for k, r in enumerate(ref["trajectory"]))
    log(f"cfg1 pulay: {len(hist)} iterations (oracle {ref['n_iter']}), dF {dF:.2e} dlam(occ) {dlam:.2e} "
        f"max trajectory dF {dev:.2e}")
    assert hist[-1]["residual"] < ref["tol"]
    assert dF <= 1e-9
    assert dlam <= 1e-8
    assert abs(len(hist) - ref["n_iter"]) <= 2
    for k, r in enumerate(ref["trajectory"]):
        fk = hist[k]["free_energy"] / s.n_atoms
        assert abs(fk - r["free_per_atom"]) <= 1e-8, (k, fk, r["free_per_atom"])
        assert abs(hist[k]["residual"] - r["residual"]) <= 1e-8 * max(1.0, r["residual"]), k
    rho = to_np(out["rho_out"])
    idx = np.array(ref["rho_out_samples"]["index"])
    val = np.array(ref["rho_out_samples"]["value"])
    assert np.max(np.abs(rho[idx] - val)) <= 1e-8 * np.max(np.abs(val))
