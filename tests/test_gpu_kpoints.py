"""GPU parity of the Bloch k-point path (Sec. 2.1: Bloch-periodic orbitals,
Brillouin-zone sampling) against the oracle's native complex arithmetic.

The GPU stores a complex orbital z = u + i v as one real column [u; v] and
works on blocks closed under z -> i z (columns [u; v], [-v; u]), so every
Bloch eigenvalue appears twice; comparisons use what is unique: H_k z
element by element, filtered blocks, Ritz values (each twice), the density
of the span, energies and residuals.  Bars: FP64 results to 1e-12 relative
(1e-10 after a degree-7 filter, whose growth amplifies rounding), Ritz
values to 1e-10, the k-point SCF per iteration to 1e-8 (as the Gamma SCF)."""
import numpy as np
import pytest

import workloads as W
from oracle import kpoints, scf

from gpu_helpers import log, ragged_system, rel_err, require_gpu, small_images_system, to_np

pytestmark = pytest.mark.gpu


def _to_block(torch, Z, dtype=None):
    B = np.concatenate([np.real(Z), np.imag(Z)], axis=1)
    return torch.as_tensor(B, dtype=dtype or torch.float64).cuda().contiguous()


def _from_block(B, nd):
    B = to_np(B).astype(np.float64)
    return B[:, :nd] + 1j * B[:, nd:]


def _ctx_with_veff(torch, s, seed):
    from paper_2005_10431_amd import Context
    ctx = Context(s)
    v = np.random.default_rng(seed).uniform(-1.0, 1.0, s.nd)
    ctx.set_veff(torch.from_numpy(v).cuda())
    return ctx, v


def _rand_Z(s, n, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(-0.5, 0.5, (n, s.nd)) + 1j * rng.uniform(-0.5, 0.5, (n, s.nd))


@pytest.mark.parametrize("which", ["ragged", "images"])
def test_apply_H_k_matches_oracle(which):
    torch = require_gpu()
    s = ragged_system(n_states=6) if which == "ragged" else small_images_system(n_states=6)
    k = np.array([0.41, -0.27, 0.63])
    log(f"apply_H_k {which}: grid {s.n}, k {k}")
    ctx, v = _ctx_with_veff(torch, s, 21)
    try:
        Z = _rand_Z(s, 5, 22)
        X = _to_block(torch, Z)
        Y = torch.empty_like(X)
        ctx.apply_H_k(k, X, Y)
        ref = kpoints.apply_H_k(s, v, kpoints.projectors_k(s, k), Z, k)
        assert rel_err(_from_block(Y, s.nd), ref) <= 1e-12
        # FP32 block
        X32 = _to_block(torch, Z, torch.float32)
        Y32 = torch.empty_like(X32)
        ctx.apply_H_k(k, X32, Y32)
        Z32 = _from_block(X32, s.nd)
        ref32 = kpoints.apply_H_k(s, v, kpoints.projectors_k(s, k), Z32, k)
        assert rel_err(_from_block(Y32, s.nd), ref32) <= 2e-6
    finally:
        ctx.close()


def test_apply_and_filter_k_without_projectors():
    """Local part only (no nonlocal term): the correction pass adds only the
    boundary phases."""
    torch = require_gpu()
    s = ragged_system(nonlocal_part=False, n_states=6)
    k = np.array([0.25, 0.5, -0.75])
    ctx, v = _ctx_with_veff(torch, s, 31)
    try:
        Z = _rand_Z(s, 5, 32)
        X = _to_block(torch, Z)
        Y = torch.empty_like(X)
        ctx.apply_H_k(k, X, Y)
        assert rel_err(_from_block(Y, s.nd), kpoints.apply_H_k(s, v, [], Z, k)) <= 1e-12
        lo, hi = ctx.spectrum_bounds_k(k)
        lo_r, hi_r = kpoints.spectrum_bounds_k(s, v, [])
        assert abs(lo - lo_r) <= 1e-10 and abs(hi - hi_r) <= 1e-10
        Wk = torch.empty_like(X)
        ctx.chebyshev_filter_k(k, X, Wk, 5, lo + 0.3 * (hi - lo), hi, lo)
        ref = kpoints.chebyshev_filter_k(s, v, [], Z, k, 5, lo + 0.3 * (hi - lo), hi, lo)
        assert rel_err(_from_block(X, s.nd), ref) <= 1e-10
    finally:
        ctx.close()


def test_padded_blocks_take_the_per_point_kernel():
    """With ldx > 2 N_d the Bloch step runs the per-point kernel (the
    unpadded path reuses the Gamma local sweep): same results."""
    torch = require_gpu()
    s = small_images_system(n_states=6)
    k = np.array([-0.33, 0.71, 0.12])
    ctx, v = _ctx_with_veff(torch, s, 27)
    try:
        pk = kpoints.projectors_k(s, k)
        Z = _rand_Z(s, 4, 28)
        Xp = torch.zeros((4, 2 * s.nd + 64), dtype=torch.float64, device="cuda")
        Xp[:, : 2 * s.nd] = _to_block(torch, Z)
        Yp = torch.zeros_like(Xp)
        ctx.apply_H_k(k, Xp, Yp)
        ref = kpoints.apply_H_k(s, v, pk, Z, k)
        assert rel_err(_from_block(Yp[:, : 2 * s.nd], s.nd), ref) <= 1e-12
        lo, hi = kpoints.spectrum_bounds_k(s, v, pk)
        Wp = torch.zeros_like(Xp)
        ctx.chebyshev_filter_k(k, Xp, Wp, 6, lo + 0.5 * (hi - lo), hi, lo)
        fref = kpoints.chebyshev_filter_k(s, v, pk, Z, k, 6, lo + 0.5 * (hi - lo), hi, lo)
        assert rel_err(_from_block(Xp[:, : 2 * s.nd], s.nd), fref) <= 1e-10
    finally:
        ctx.close()


def test_apply_H_k_at_gamma_equals_the_gamma_operator():
    torch = require_gpu()
    s = ragged_system(n_states=6)
    ctx, v = _ctx_with_veff(torch, s, 23)
    try:
        Z = _rand_Z(s, 3, 24)
        X = _to_block(torch, Z)
        Y = torch.empty_like(X)
        ctx.apply_H_k([0.0, 0.0, 0.0], X, Y)
        R = torch.as_tensor(np.real(Z)).cuda().contiguous()
        I = torch.as_tensor(np.imag(Z)).cuda().contiguous()
        HR, HI = torch.empty_like(R), torch.empty_like(I)
        ctx.apply_H(R, HR)
        ctx.apply_H(I, HI)
        got = _from_block(Y, s.nd)
        ref = to_np(HR) + 1j * to_np(HI)
        assert rel_err(got, ref) <= 1e-12
    finally:
        ctx.close()


def test_filter_rr_and_bounds_k_match_oracle():
    torch = require_gpu()
    from paper_2005_10431_amd.driver import bloch_block
    s = small_images_system(n_states=6)
    k = np.array([0.9, 0.2, -0.5])
    ctx, v = _ctx_with_veff(torch, s, 25)
    try:
        pk = kpoints.projectors_k(s, k)
        lo, hi = ctx.spectrum_bounds_k(k)
        lo_r, hi_r = kpoints.spectrum_bounds_k(s, v, pk)
        assert abs(lo - lo_r) <= 1e-10 and abs(hi - hi_r) <= 1e-10
        Z = _rand_Z(s, 5, 26)
        # filter on plain columns
        X = _to_block(torch, Z)
        Wk = torch.empty_like(X)
        a, b, a0 = lo_r + 0.4 * (hi_r - lo_r), hi_r, lo_r
        ctx.chebyshev_filter_k(k, X, Wk, 7, a, b, a0)
        ref = kpoints.chebyshev_filter_k(s, v, pk, Z, k, 7, a, b, a0)
        assert rel_err(_from_block(X, s.nd), ref) <= 1e-10
        # Rayleigh-Ritz on the z -> i z closed block
        B = bloch_block(Z, torch.float64)
        eig = torch.empty(10, dtype=torch.float64, device="cuda")
        ctx.rayleigh_ritz_k(k, B, eig)
        Xr, lam = kpoints.rayleigh_ritz_k(s, v, pk, Z, k)
        e = to_np(eig)
        np.testing.assert_allclose(e[0::2], lam, atol=1e-10)
        np.testing.assert_allclose(e[1::2], lam, atol=1e-10)
        Bn = to_np(B)
        dens_gpu = np.sum(Bn[:, :s.nd] ** 2 + Bn[:, s.nd:] ** 2, axis=0)
        dens_ref = 2.0 * np.sum(np.abs(Xr) ** 2, axis=0)
        assert rel_err(dens_gpu, dens_ref) <= 1e-10
    finally:
        ctx.close()


def test_k_point_scf_matches_oracle():
    """Two k-points (a 2 x 1 x 1 Monkhorst-Pack set) on the small ragged
    cell with projectors: the first iterations follow the oracle's k-point
    SCF, and the converged free energy and spectra agree."""
    require_gpu()
    from paper_2005_10431_amd.driver import run_scf_k
    s = W.tiny_system(n=(14, 16, 18), n_states=8)
    kpts, wk = W.monkhorst_pack(s.L, (2, 1, 1))
    Z0 = [W.initial_orbitals_k(s.nd, s.n_states, s.seed, q) for q in range(len(kpts))]
    ref = kpoints.scf_k(s, kpts, wk, Z0, max_iter=200, tol=1e-10)
    out = run_scf_k(s, kpts, wk, Z0, max_iter=200, tol=1e-10)
    h, hr = out["history"], ref["history"]
    log(f"k-point SCF: {len(h)} iterations (oracle {len(hr)}), F {h[-1]['free_energy']:.12f} "
        f"(oracle {hr[-1]['free']:.12f})")
    for k in range(min(8, len(hr))):
        assert abs(h[k]["free_energy"] - hr[k]["free"]) <= 1e-8, k
        assert abs(h[k]["residual"] - hr[k]["residual"]) <= 1e-8 * max(1.0, hr[k]["residual"]), k
    assert h[-1]["residual"] < 1e-10
    assert abs(h[-1]["free_energy"] - hr[-1]["free"]) <= 1e-9
    assert abs(len(h) - len(hr)) <= 2
    for q in range(len(kpts)):
        g = ref["g"][q] > 1e-4
        np.testing.assert_allclose(h[-1]["eig_k"][q][g], ref["lam"][q][g], atol=1e-8)
    out["ctx"].close()


def test_k_state_rejects_bad_weights():
    torch = require_gpu()
    from paper_2005_10431_amd import Context, SparcError, make_k_state
    s = small_images_system(n_states=4)
    ctx = Context(s)
    try:
        B = torch.zeros((8, 2 * s.nd), dtype=torch.float64, device="cuda")
        rho = torch.ones(s.nd, dtype=torch.float64, device="cuda")
        eig = torch.zeros(16, dtype=torch.float64, device="cuda")
        occ = torch.zeros_like(eig)
        st = make_k_state(rho, [B, B.clone()], np.zeros((2, 3)), [0.7, 0.7], eig, occ, 8)
        with pytest.raises(SparcError) as e:
            ctx.scf_step_k(st)
        assert e.value.status == 1
        with pytest.raises(SparcError):
            ctx.apply_H_k([0.1, 0.0, 0.0], B[:, : s.nd].contiguous(), B.clone()[:, : s.nd].contiguous())
    finally:
        ctx.close()


def test_filter_k_fp32_and_k_point_scf_fp32():
    """FP32 Bloch blocks: the filter against the oracle on the same
    FP32-rounded input (bar 2e-5 relative after degree 7, FP32 rounding
    of every step), and the FP32 k-point SCF converged to 1e-5 within 1e-5
    Ha/atom of the oracle's FP64 fixed point."""
    torch = require_gpu()
    from paper_2005_10431_amd.driver import run_scf_k
    s = small_images_system(n_states=6)
    k = np.array([0.5, -0.25, 0.75])
    ctx, v = _ctx_with_veff(torch, s, 29)
    try:
        pk = kpoints.projectors_k(s, k)
        lo, hi = kpoints.spectrum_bounds_k(s, v, pk)
        X = _to_block(torch, _rand_Z(s, 4, 30), torch.float32)
        Z32 = _from_block(X, s.nd)
        Wk = torch.empty_like(X)
        a = lo + 0.4 * (hi - lo)
        ctx.chebyshev_filter_k(k, X, Wk, 7, a, hi, lo)
        ref = kpoints.chebyshev_filter_k(s, v, pk, Z32, k, 7, a, hi, lo)
        assert rel_err(_from_block(X, s.nd), ref) <= 2e-5
    finally:
        ctx.close()
    s2 = W.tiny_system(n=(14, 16, 18), n_states=8)
    kpts, wk = W.monkhorst_pack(s2.L, (2, 1, 1))
    Z0 = [W.initial_orbitals_k(s2.nd, s2.n_states, s2.seed, q) for q in range(len(kpts))]
    ref = kpoints.scf_k(s2, kpts, wk, Z0, max_iter=200, tol=1e-10)
    out = run_scf_k(s2, kpts, wk, Z0, prec="fp32", max_iter=200, tol=1e-5)
    h = out["history"]
    dF = abs(h[-1]["free_energy"] - ref["history"][-1]["free"]) / s2.n_atoms
    log(f"k-point SCF FP32: {len(h)} iterations, dF/atom {dF:.2e}")
    assert h[-1]["residual"] < 1e-5
    assert dF <= 1e-5
    out["ctx"].close()


def test_k_point_scf_with_pulay_and_kerker_matches_oracle():
    """Two k-points with restarted periodic Pulay mixing (history 7, period
    2) and the Kerker-type preconditioner: trajectory and fixed point
    against the oracle."""
    require_gpu()
    from dataclasses import replace
    from paper_2005_10431_amd.driver import run_scf_k
    s = replace(W.tiny_system(n=(14, 16, 18), n_states=8), pulay_history=7, pulay_period=2, pulay_restart=1,
                kerker_q0=1.0)
    kpts, wk = W.monkhorst_pack(s.L, (2, 1, 1))
    Z0 = [W.initial_orbitals_k(s.nd, s.n_states, s.seed, q) for q in range(len(kpts))]
    ref = kpoints.scf_k(s, kpts, wk, Z0, max_iter=200, tol=1e-10)
    out = run_scf_k(s, kpts, wk, Z0, max_iter=200, tol=1e-10)
    h, hr = out["history"], ref["history"]
    log(f"k-point Pulay SCF: {len(h)} iterations (oracle {len(hr)})")
    for k in range(min(8, len(hr))):
        assert abs(h[k]["free_energy"] - hr[k]["free"]) <= 1e-8, k
    assert h[-1]["residual"] < 1e-10
    assert abs(h[-1]["free_energy"] - hr[-1]["free"]) <= 1e-9
    assert abs(len(h) - len(hr)) <= 2
    out["ctx"].close()
