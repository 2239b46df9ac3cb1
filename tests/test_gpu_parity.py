"""GPU <-> oracle parity of every step of the hot path, through the C ABI.

Tolerances (FP64): 1e-12 relative on one H.X, 1e-8 Ha on eigenvalues,
1e-6 Ha/atom on the free energy.  FP32 blocks: relative errors of the order
of single-precision rounding of the stencil sum (1e-5).
"""
import numpy as np
import pytest

import workloads as W
from oracle import atoms, chefsi, electrostatics, hamiltonian, scf, xc

from gpu_helpers import (log, ragged_system, rel_err, require_gpu, small_images_system, to_dev, to_np)

pytestmark = pytest.mark.gpu


def _ctx(system):
    from paper_2005_10431_amd import Context
    return Context(system)


def _veff(system, seed=11, scale=0.5):
    return np.random.default_rng(seed).uniform(-scale, scale, system.nd)


@pytest.mark.parametrize("make", [ragged_system, small_images_system], ids=["ragged", "images"])
def test_apply_H_fp64(make):
    torch = require_gpu()
    s = make()
    log("apply_H fp64", s.n, s.L)
    ctx = _ctx(s)
    projs = atoms.projectors(s)
    v = _veff(s)
    X = W.initial_orbitals(s.nd, 5, 1)
    Yref = hamiltonian.apply_H(s, v, projs, X)
    ctx.set_veff(to_dev(torch, v))
    Xd = to_dev(torch, X)
    Yd = torch.zeros_like(Xd)
    ctx.apply_H(Xd, Yd)
    Y = to_np(Yd)
    assert rel_err(Y, Yref) <= 1e-12
    assert np.max(np.abs(Y - Yref)) <= 1e-12 * np.max(np.abs(Yref))


def test_apply_H_fp64_padded_leading_dimension():
    torch = require_gpu()
    s = ragged_system()
    ctx = _ctx(s)
    projs = atoms.projectors(s)
    v = _veff(s, 12)
    X = W.initial_orbitals(s.nd, 3, 2)
    ld = s.nd + 37
    Xp = np.zeros((3, ld))
    Xp[:, :s.nd] = X
    ctx.set_veff(to_dev(torch, v))
    Xd = to_dev(torch, Xp)
    Yd = torch.full_like(Xd, 7.0)
    ctx.apply_H(Xd, Yd)
    Y = to_np(Yd)
    Yref = hamiltonian.apply_H(s, v, projs, X)
    assert rel_err(Y[:, :s.nd], Yref) <= 1e-12
    assert np.all(Y[:, s.nd:] == 7.0)          # padding untouched


def test_apply_H_fp32():
    torch = require_gpu()
    s = ragged_system()
    ctx = _ctx(s)
    projs = atoms.projectors(s)
    v = _veff(s)
    X = W.initial_orbitals(s.nd, 4, 3).astype(np.float32)
    Yref = hamiltonian.apply_H(s, v, projs, X.astype(np.float64))
    ctx.set_veff(to_dev(torch, v))
    Xd = to_dev(torch, X)
    Yd = torch.zeros_like(Xd)
    ctx.apply_H(Xd, Yd)
    assert rel_err(to_np(Yd).astype(np.float64), Yref) <= 2e-6


def test_apply_H_cfg2_sampled_columns():
    """Full config-2 block (72^3, 260 states, 108 atoms with s+p projectors)
    in the launch configuration of the benchmark; the oracle recomputes three
    columns one by one."""
    torch = require_gpu()
    s = W.config2(0)
    log("apply_H cfg2 full block")
    ctx = _ctx(s)
    v = _veff(s, 21, 1.0)
    X = W.initial_orbitals(s.nd, s.n_states, 0)
    ctx.set_veff(to_dev(torch, v))
    Xd = to_dev(torch, X)
    Yd = torch.zeros_like(Xd)
    ctx.apply_H(Xd, Yd)
    torch.cuda.synchronize()
    projs = atoms.projectors(s)
    for j in (0, 137, 259):
        yref = hamiltonian.apply_H(s, v, projs, X[j:j + 1])[0]
        y = to_np(Yd[j])
        assert rel_err(y, yref) <= 1e-12, j


@pytest.mark.parametrize("degree", [1, 7, 8])
def test_chebyshev_filter_fp64(degree):
    torch = require_gpu()
    s = small_images_system()
    ctx = _ctx(s)
    projs = atoms.projectors(s)
    v = _veff(s, 13)
    lo, hi = hamiltonian.spectrum_bounds(s, v, projs)
    a, b, a0 = lo + 0.3 * (hi - lo), hi, lo
    X = W.initial_orbitals(s.nd, 6, 4)
    Yref = chefsi.chebyshev_filter(s, v, projs, X, degree, a, b, a0)
    ctx.set_veff(to_dev(torch, v))
    Xd = to_dev(torch, X)
    Wd = torch.zeros_like(Xd)
    ctx.chebyshev_filter(Xd, Wd, degree, a, b, a0)
    assert rel_err(to_np(Xd), Yref) <= 1e-11


def test_chebyshev_filter_cfg2_sampled_columns():
    """Degree-20 filter over the full config-2 block; the filter acts column
    by column, so the oracle filters two columns alone."""
    torch = require_gpu()
    s = W.config2(0)
    log("filter cfg2 full block")
    ctx = _ctx(s)
    projs = atoms.projectors(s)
    v = _veff(s, 22, 1.0)
    lo, hi = hamiltonian.spectrum_bounds(s, v, projs)
    a, b, a0 = lo + 0.05 * (hi - lo), hi, lo
    X = W.initial_orbitals(s.nd, s.n_states, 1)
    ctx.set_veff(to_dev(torch, v))
    Xd = to_dev(torch, X)
    Wd = torch.empty_like(Xd)
    ctx.chebyshev_filter(Xd, Wd, 20, a, b, a0)
    torch.cuda.synchronize()
    for j in (3, 258):
        yref = chefsi.chebyshev_filter(s, v, projs, X[j:j + 1], 20, a, b, a0)[0]
        assert rel_err(to_np(Xd[j]), yref) <= 1e-11, j


# FP32 filter bar: each of the m sweeps commits at most the rounding of one
# FP32 stencil application (the H X bar of 2e-6 relative, test_apply_H_fp32),
# errors add at worst linearly, and the scaled recurrence keeps every iterate
# within the norm of its input; a factor 2 covers the recurrence term.
def fp32_filter_bar(m):
    return 2.0 * m * 2e-6


@pytest.mark.parametrize("make", [ragged_system, small_images_system], ids=["ragged", "images"])
@pytest.mark.parametrize("degree", [7, 8])
def test_chebyshev_filter_fp32_nonlocal(make, degree):
    """FP32 filter with s+p projectors (the nonlocal sweep in its first-step
    and later-step forms, odd and even degree) against the oracle filtering
    the same FP32-rounded block in FP64."""
    torch = require_gpu()
    s = make()
    log("filter fp32 nonlocal", s.n, "degree", degree)
    ctx = _ctx(s)
    projs = atoms.projectors(s)
    v = _veff(s, 23)
    lo, hi = hamiltonian.spectrum_bounds(s, v, projs)
    a, b, a0 = lo + 0.3 * (hi - lo), hi, lo
    X = W.initial_orbitals(s.nd, 6, 9).astype(np.float32)
    Yref = chefsi.chebyshev_filter(s, v, projs, X.astype(np.float64), degree, a, b, a0)
    ctx.set_veff(to_dev(torch, v))
    Xd = to_dev(torch, X)
    Wd = torch.zeros_like(Xd)
    ctx.chebyshev_filter(Xd, Wd, degree, a, b, a0)
    err = rel_err(to_np(Xd).astype(np.float64), Yref)
    log(f"  rel err {err:.2e} (bar {fp32_filter_bar(degree):.1e})")
    assert err <= fp32_filter_bar(degree)


def test_chebyshev_filter_fp32_cfg2_sampled_columns():
    """Degree-20 FP32 filter over the full config-2 block with projectors, in
    the launch configuration of the benchmark; the oracle filters two of the
    FP32-rounded columns alone in FP64."""
    torch = require_gpu()
    s = W.config2(0)
    log("filter fp32 cfg2 full block")
    ctx = _ctx(s)
    projs = atoms.projectors(s)
    v = _veff(s, 24, 1.0)
    lo, hi = hamiltonian.spectrum_bounds(s, v, projs)
    a, b, a0 = lo + 0.05 * (hi - lo), hi, lo
    X = W.initial_orbitals(s.nd, s.n_states, 3).astype(np.float32)
    ctx.set_veff(to_dev(torch, v))
    Xd = to_dev(torch, X)
    Wd = torch.empty_like(Xd)
    ctx.chebyshev_filter(Xd, Wd, s.cheb_degree, a, b, a0)
    torch.cuda.synchronize()
    for j in (5, 259):
        yref = chefsi.chebyshev_filter(s, v, projs, X[j:j + 1].astype(np.float64), s.cheb_degree, a, b, a0)[0]
        err = rel_err(to_np(Xd[j]).astype(np.float64), yref)
        log(f"  column {j}: rel err {err:.2e}")
        assert err <= fp32_filter_bar(s.cheb_degree), j


def _projector(X, dV):
    return dV * X.T @ X


def test_rayleigh_ritz_fp64():
    torch = require_gpu()
    s = small_images_system(n_states=8)
    ctx = _ctx(s)
    projs = atoms.projectors(s)
    v = _veff(s, 14)
    X = W.initial_orbitals(s.nd, 8, 5)
    Xr, lam = chefsi.rayleigh_ritz(s, v, projs, X)
    ctx.set_veff(to_dev(torch, v))
    Xd = to_dev(torch, X)
    eig = torch.zeros(8, dtype=torch.float64, device="cuda")
    ctx.rayleigh_ritz(Xd, eig)
    Xg = to_np(Xd)
    np.testing.assert_allclose(to_np(eig), lam, atol=1e-10)
    O = s.dV * Xg @ Xg.T
    assert np.max(np.abs(O - np.eye(8))) < 1e-12
    # same Ritz subspace, column by column up to sign (eigenvalues are simple)
    for j in range(8):
        c = s.dV * float(Xg[j] @ Xr[j])
        assert abs(abs(c) - 1.0) < 1e-9, j


@pytest.mark.parametrize("tile", ["by_size", "160"])
def test_rayleigh_ritz_wide_block(tile, monkeypatch):
    """400 columns: above the size from which the Gram and projected-H
    products use 128-wide tiles (checked against the 160-wide tiles too)."""
    torch = require_gpu()
    ncol = 400
    if tile != "by_size":
        monkeypatch.setenv("SPARC_GPU_GEMM_TILE", tile)
    s = small_images_system(n_states=ncol)
    log("rayleigh_ritz wide block", ncol, "tile", tile)
    ctx = _ctx(s)
    projs = atoms.projectors(s)
    v = _veff(s, 16)
    X = W.initial_orbitals(s.nd, ncol, 6)
    Xr, lam = chefsi.rayleigh_ritz(s, v, projs, X)
    ctx.set_veff(to_dev(torch, v))
    Xd = to_dev(torch, X)
    eig = torch.zeros(ncol, dtype=torch.float64, device="cuda")
    ctx.rayleigh_ritz(Xd, eig)
    Xg = to_np(Xd)
    scale = max(1.0, float(np.max(np.abs(lam))))
    np.testing.assert_allclose(to_np(eig), lam, atol=1e-10 * scale)
    O = s.dV * Xg @ Xg.T
    assert np.max(np.abs(O - np.eye(ncol))) < 1e-11
    # the lowest 20 Ritz vectors span the oracle's (projector difference)
    P = s.dV * Xg[:20].T @ Xg[:20]
    Pr = s.dV * Xr[:20].T @ Xr[:20]
    assert np.max(np.abs(P - Pr)) < 1e-8


def test_rayleigh_ritz_fp32():
    torch = require_gpu()
    s = small_images_system(n_states=8)
    ctx = _ctx(s)
    projs = atoms.projectors(s)
    v = _veff(s, 14)
    X = W.initial_orbitals(s.nd, 8, 5)
    _, lam = chefsi.rayleigh_ritz(s, v, projs, X)
    ctx.set_veff(to_dev(torch, v))
    Xd = to_dev(torch, X, torch.float32)
    eig = torch.zeros(8, dtype=torch.float64, device="cuda")
    ctx.rayleigh_ritz(Xd, eig)
    np.testing.assert_allclose(to_np(eig), lam, atol=2e-4 * np.max(np.abs(lam)))
    Xg = to_np(Xd).astype(np.float64)
    assert np.max(np.abs(s.dV * Xg @ Xg.T - np.eye(8))) < 1e-5


def _span_sines(s, Xg, Xr, k):
    """Sines of the principal angles between the spans of the first k rows."""
    cos = np.linalg.svd(s.dV * Xg[:k] @ Xr[:k].T, compute_uv=False)
    return np.sqrt(np.maximum(0.0, 1.0 - np.minimum(cos, 1.0) ** 2))


@pytest.mark.parametrize("ncol, tile", [(400, "by_size"), (400, "160"), (1200, "by_size")])
def test_rayleigh_ritz_fp32_wide_block(ncol, tile, monkeypatch):
    """FP32 Rayleigh-Ritz at the subspace sizes of the benchmark workloads:
    Gram and projected H on FP32 MFMA tiles (128-wide above N = 320, and the
    160-wide tiles at 400 columns) with split-K partials reduced in FP64,
    FP64 Cholesky and eigensolver, FP32 rotation.  Against the oracle's FP64
    Rayleigh-Ritz of the same FP32-rounded block:
      - Ritz values within 2e-4 max|lambda| (the 8-column FP32 bar);
      - dV X^T X = I within 1e-5 (FP32 rounding of the rotated block);
      - the lowest k states span the oracle's subspace, k at the widest
        spectral gap between 20 and 60: by the Davis-Kahan bound the sines of
        the principal angles stay below 2 delta / gap, delta the Ritz bar."""
    torch = require_gpu()
    if tile != "by_size":
        monkeypatch.setenv("SPARC_GPU_GEMM_TILE", tile)
    s = small_images_system(n_states=ncol) if ncol <= 400 else ragged_system(n_states=ncol)
    log("rayleigh_ritz fp32", ncol, "columns, tile", tile, "grid", s.n)
    ctx = _ctx(s)
    projs = atoms.projectors(s)
    v = _veff(s, 19)
    X = W.initial_orbitals(s.nd, ncol, 11).astype(np.float32)
    Xr, lam = chefsi.rayleigh_ritz(s, v, projs, X.astype(np.float64))
    ctx.set_veff(to_dev(torch, v))
    Xd = to_dev(torch, X)
    eig = torch.zeros(ncol, dtype=torch.float64, device="cuda")
    ctx.rayleigh_ritz(Xd, eig)
    Xg = to_np(Xd).astype(np.float64)
    delta = 2e-4 * float(np.max(np.abs(lam)))
    dl = np.max(np.abs(to_np(eig) - lam))
    O = s.dV * Xg @ Xg.T
    orth = np.max(np.abs(O - np.eye(ncol)))
    gaps = lam[21:61] - lam[20:60]
    k = 21 + int(np.argmax(gaps))
    gap = float(np.max(gaps))
    sines = _span_sines(s, Xg, Xr, k)
    log(f"  max|dlam| {dl:.2e} (bar {delta:.2e}), orthonormality {orth:.2e}, span k={k} gap {gap:.3e} "
        f"max sin {np.max(sines):.2e}")
    assert dl <= delta
    assert orth <= 1e-5
    assert np.max(sines) <= min(1.0, 2.0 * delta / gap)


def test_rayleigh_ritz_1200_columns():
    """The cfg4 subspace size on a 40 x 37 x 13 grid: Gram and projected H
    on 128-wide tiles, Cholesky and tridiagonalisation over many workgroups,
    all against the oracle."""
    torch = require_gpu()
    ncol = 1200
    s = ragged_system(n_states=ncol)
    log("rayleigh_ritz", ncol, "columns on", s.n)
    ctx = _ctx(s)
    projs = atoms.projectors(s)
    v = _veff(s, 18)
    X = W.initial_orbitals(s.nd, ncol, 7)
    Xr, lam = chefsi.rayleigh_ritz(s, v, projs, X)
    ctx.set_veff(to_dev(torch, v))
    Xd = to_dev(torch, X)
    eig = torch.zeros(ncol, dtype=torch.float64, device="cuda")
    ctx.rayleigh_ritz(Xd, eig)
    Xg = to_np(Xd)
    scale = max(1.0, float(np.max(np.abs(lam))))
    np.testing.assert_allclose(to_np(eig), lam, atol=1e-10 * scale)
    O = s.dV * Xg @ Xg.T
    assert np.max(np.abs(O - np.eye(ncol))) < 1e-10
    # lowest 40 Ritz vectors: the same subspace (all principal cosines 1)
    cos = np.linalg.svd(s.dV * Xg[:40] @ Xr[:40].T, compute_uv=False)
    assert 1.0 - np.min(cos) < 1e-9


def test_cholesky_over_many_workgroups_is_bitwise_identical(monkeypatch):
    """From N = 384 the Cholesky factor's trailing updates run over many
    workgroups; each entry gets the same operations in the same order as in
    the one-workgroup kernel, so the Rayleigh-Ritz results are bitwise
    equal."""
    torch = require_gpu()
    ncol = 400
    s = small_images_system(n_states=ncol)
    v = _veff(s, 17)
    X = W.initial_orbitals(s.nd, ncol, 8)
    out = {}
    for name, threshold in (("one workgroup", 1 << 30), ("many workgroups", 384)):
        monkeypatch.setenv("SPARC_GPU_CHOL_MULTI_MIN", str(threshold))
        log("rayleigh_ritz", ncol, "cholesky", name)
        ctx = _ctx(s)
        ctx.set_veff(to_dev(torch, v))
        Xd = to_dev(torch, X)
        eig = torch.zeros(ncol, dtype=torch.float64, device="cuda")
        ctx.rayleigh_ritz(Xd, eig)
        out[name] = (to_np(eig), to_np(Xd))
        ctx.close()
    np.testing.assert_array_equal(out["one workgroup"][0], out["many workgroups"][0])
    np.testing.assert_array_equal(out["one workgroup"][1], out["many workgroups"][1])


def test_rayleigh_ritz_rank_deficient_wide_block():
    """The many-workgroup Cholesky reports a rank-deficient block too."""
    from paper_2005_10431_amd import SparcError
    torch = require_gpu()
    ncol = 400
    s = small_images_system(n_states=ncol)
    ctx = _ctx(s)
    ctx.set_veff(to_dev(torch, _veff(s)))
    X = W.initial_orbitals(s.nd, ncol, 9)
    X[350] = X[10]
    Xd = to_dev(torch, X)
    eig = torch.zeros(ncol, dtype=torch.float64, device="cuda")
    with pytest.raises(SparcError) as ei:
        ctx.rayleigh_ritz(Xd, eig)
    assert ei.value.name == "SPARC_ERR_NOT_SPD"
    np.testing.assert_array_equal(to_np(Xd), X)


def test_rayleigh_ritz_rank_deficient_block():
    from paper_2005_10431_amd import SparcError
    torch = require_gpu()
    s = small_images_system(n_states=4)
    ctx = _ctx(s)
    ctx.set_veff(to_dev(torch, _veff(s)))
    X = W.initial_orbitals(s.nd, 4, 6)
    X[3] = X[1]
    Xd = to_dev(torch, X)
    eig = torch.zeros(4, dtype=torch.float64, device="cuda")
    with pytest.raises(SparcError) as ei:
        ctx.rayleigh_ritz(Xd, eig)
    assert ei.value.name == "SPARC_ERR_NOT_SPD"
    np.testing.assert_array_equal(to_np(Xd), X)


def test_occupations_and_density():
    torch = require_gpu()
    s = W.config1(0)
    ctx = _ctx(s)
    lam = np.sort(np.random.default_rng(8).uniform(-0.6, 0.3, s.n_states))
    mu_ref, g_ref = scf.occupations(lam, s.n_electrons, s.kT)
    eig = to_dev(torch, lam)
    occ = torch.zeros_like(eig)
    mu = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.occupations(eig, occ, mu)
    np.testing.assert_allclose(to_np(occ), g_ref, atol=1e-12)
    assert abs(float(to_np(mu)[0]) - mu_ref) < 1e-10
    X = W.initial_orbitals(s.nd, s.n_states, 7)
    rho = torch.zeros(s.nd, dtype=torch.float64, device="cuda")
    ctx.density(to_dev(torch, X), occ, rho)
    assert rel_err(to_np(rho), scf.density(X, g_ref)) <= 1e-13


@pytest.mark.parametrize("make", [W.config1, small_images_system], ids=["cfg1", "images"])
def test_pseudocharge_energies_and_sad(make):
    torch = require_gpu()
    s = make()
    ctx = _ctx(s)
    b = torch.zeros(s.nd, dtype=torch.float64, device="cuda")
    es, ec = ctx.pseudocharge(b)
    assert rel_err(to_np(b), atoms.pseudocharge(s)) <= 1e-13
    assert abs(es - atoms.self_energy(s)) <= 1e-11 * abs(es)
    assert abs(ec - atoms.overlap_correction(s)) <= 1e-12 * max(1.0, abs(ec))
    rho = torch.zeros(s.nd, dtype=torch.float64, device="cuda")
    ctx.sad_density(rho)
    assert rel_err(to_np(rho), atoms.sad_density(s)) <= 1e-13


def test_potential_matches_oracle():
    torch = require_gpu()
    s = W.config1(0)
    ctx = _ctx(s)
    st = scf.setup(s)
    rho = atoms.sad_density(s)
    phi, exc, vxc, veff = scf.potential(s, st, rho)
    d = lambda: torch.zeros(s.nd, dtype=torch.float64, device="cuda")
    P, E, V, VE = d(), d(), d(), d()
    ctx.potential(to_dev(torch, rho), P, E, V, VE)
    assert np.max(np.abs(to_np(P) - phi)) <= 1e-11 * max(1.0, np.max(np.abs(phi)))
    assert rel_err(to_np(E), exc) <= 1e-13
    assert rel_err(to_np(V), vxc) <= 1e-13
    assert np.max(np.abs(to_np(VE) - veff)) <= 1e-11 * max(1.0, np.max(np.abs(veff)))


def test_spectrum_bounds_match_oracle():
    torch = require_gpu()
    s = small_images_system()
    ctx = _ctx(s)
    v = _veff(s, 15)
    ctx.set_veff(to_dev(torch, v))
    lo, hi = ctx.spectrum_bounds()
    lo_r, hi_r = hamiltonian.spectrum_bounds(s, v, atoms.projectors(s))
    assert abs(lo - lo_r) < 1e-11 and abs(hi - hi_r) < 1e-10


def test_argument_errors():
    from paper_2005_10431_amd import SparcError
    torch = require_gpu()
    s = small_images_system(n_states=4)
    ctx = _ctx(s)
    X = torch.zeros((4, s.nd), dtype=torch.float64, device="cuda")
    Y = torch.zeros_like(X)
    with pytest.raises(SparcError, match="SPARC_ERR_ARG"):
        ctx.apply_H(X, X)                              # aliasing
    with pytest.raises(SparcError, match="SPARC_ERR_ARG"):
        ctx.chebyshev_filter(X, Y, 5, 1.0, 2.0, 3.0)   # a0 >= a
    big = torch.zeros((5, s.nd), dtype=torch.float64, device="cuda")
    with pytest.raises(SparcError, match="SPARC_ERR_ARG"):
        ctx.apply_H(big, torch.zeros_like(big))        # ncol > n_states
    short = torch.zeros((4, s.nd - 1), dtype=torch.float64, device="cuda")
    with pytest.raises(SparcError, match="SPARC_ERR_ARG"):
        ctx.apply_H(short, torch.zeros_like(short))    # ldx < N_d
    # occupations: the electrons must fit in the states (N_e <= 2 ncol)
    ncol = int(s.n_electrons // 2) - 1
    assert ncol >= 1
    eig = torch.linspace(-1.0, 1.0, ncol, dtype=torch.float64, device="cuda")
    occ = torch.zeros_like(eig)
    with pytest.raises(SparcError, match="SPARC_ERR_ARG"):
        ctx.occupations(eig, occ)
    empty = torch.zeros(0, dtype=torch.float64, device="cuda")
    with pytest.raises(SparcError, match="SPARC_ERR_ARG"):
        ctx.occupations(empty, torch.zeros_like(empty))  # no states


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_filter_is_bitwise_reproducible(prec):
    """Every reduction of the filter has a fixed order (the projection pass:
    pair sums in segment order, each candidate's pairs in row order, planes
    in order, per-atom partials in (slab, candidate, z range) order), so two
    filters of the same block agree bit for bit, on one context and across
    contexts."""
    torch = require_gpu()
    s = ragged_system(n_states=70)
    v = _veff(s, 21)
    X = W.initial_orbitals(s.nd, s.n_states, 4)
    dt = torch.float64 if prec == "fp64" else torch.float32
    outs = []
    for rep in range(3):
        ctx = _ctx(s) if rep != 1 else ctx
        ctx.set_veff(to_dev(torch, v))
        lo, hi = ctx.spectrum_bounds()
        Xd = to_dev(torch, X, dt)
        Wd = torch.empty_like(Xd)
        ctx.chebyshev_filter(Xd, Wd, 9, 0.5 * (lo + hi), hi, lo)
        outs.append(to_np(Xd))
    log("filter reproducibility: max |diff|", float(np.max(np.abs(outs[0] - outs[1]))),
        float(np.max(np.abs(outs[0] - outs[2]))))
    assert np.array_equal(outs[0], outs[1])
    assert np.array_equal(outs[0], outs[2])


@pytest.mark.parametrize("system", ["ragged", "images"])
def test_fp64_nonlocal_slot_counts_agree_bitwise(system, monkeypatch):
    """The FP64 sweep adds 6 nonlocal slots per point when no point of its
    tables lies in more than 6 supports, else 7; forced to 7
    (SPARC_GPU_NL_SLOTS=7, read at context creation), the extra slot names
    the empty pair, adds an exact zero, and H X and the filter are bitwise
    the same."""
    torch = require_gpu()
    s = ragged_system(n_states=6) if system == "ragged" else small_images_system(n_states=6)
    v = _veff(s, 23)
    X = W.initial_orbitals(s.nd, s.n_states, 5)
    outs = []
    for force in (None, "7"):
        if force:
            monkeypatch.setenv("SPARC_GPU_NL_SLOTS", force)
        else:
            monkeypatch.delenv("SPARC_GPU_NL_SLOTS", raising=False)
        ctx = _ctx(s)
        ctx.set_veff(to_dev(torch, v))
        lo, hi = ctx.spectrum_bounds()
        Xd = to_dev(torch, X)
        Yd = torch.empty_like(Xd)
        ctx.apply_H(Xd, Yd)
        Wd = torch.empty_like(Xd)
        ctx.chebyshev_filter(Xd, Wd, 8, 0.5 * (lo + hi), hi, lo)
        outs.append((to_np(Yd), to_np(Xd)))
    monkeypatch.delenv("SPARC_GPU_NL_SLOTS", raising=False)
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])


def test_projection_over_ragged_z_ranges():
    """14 x 16 x 37 grid, 4 atoms, 4 columns: the projection pass splits the
    37 planes of each slab into 4 z ranges of 10, 10, 10 and 7 planes, whose
    partials the per-atom sum adds in order.  H X and a degree-7 filter
    against the oracle, and the allocation-free filter bitwise equal to the
    filter."""
    torch = require_gpu()
    s = W.tiny_system(n=(14, 16, 37), L=(7.0, 7.5, 11.1), n_atoms=4, seed=13, n_states=4)
    v = _veff(s, 29)
    projs = atoms.projectors(s)
    X = W.initial_orbitals(s.nd, s.n_states, 6)
    ctx = _ctx(s)
    ctx.set_veff(to_dev(torch, v))
    Xd = to_dev(torch, X)
    Yd = torch.empty_like(Xd)
    ctx.apply_H(Xd, Yd)
    torch.cuda.synchronize()
    err = rel_err(to_np(Yd), hamiltonian.apply_H(s, v, projs, X))
    log(f"ragged z ranges: H X rel err {err:.2e}")
    assert err <= 1e-12
    lo, hi = hamiltonian.spectrum_bounds(s, v, projs)
    a, b, a0 = lo + 0.3 * (hi - lo), hi, lo
    Wd = torch.empty_like(Xd)
    ctx.chebyshev_filter(Xd, Wd, 7, a, b, a0)
    X2 = to_dev(torch, X)
    W2 = torch.empty_like(X2)
    ctx.chebyshev_filter_noalloc(X2, W2, 7, a, b, a0)
    torch.cuda.synchronize()
    ref = chefsi.chebyshev_filter(s, v, projs, X, 7, a, b, a0)
    err = rel_err(to_np(Xd), ref)
    log(f"ragged z ranges: filter rel err {err:.2e}")
    assert err <= 1e-11
    assert torch.equal(Xd, X2)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_projection_workgroup_size_does_not_change_results(prec, monkeypatch):
    """The projection pass gives each orbital its own wave, so the number of
    orbitals per workgroup (SPARC_GPU_PROJ_NB=2 against the default 8, read at
    context creation) changes no sum: with one z range per slab (13 planes)
    H X and the filter are bitwise the same."""
    torch = require_gpu()
    s = ragged_system(n_states=11)
    v = _veff(s, 31)
    X = W.initial_orbitals(s.nd, s.n_states, 8)
    dt = torch.float64 if prec == "fp64" else torch.float32
    outs = []
    for nb in (None, "2"):
        if nb:
            monkeypatch.setenv("SPARC_GPU_PROJ_NB", nb)
        else:
            monkeypatch.delenv("SPARC_GPU_PROJ_NB", raising=False)
        ctx = _ctx(s)
        ctx.set_veff(to_dev(torch, v))
        lo, hi = ctx.spectrum_bounds()
        Xd = to_dev(torch, X, dt)
        Yd = torch.empty_like(Xd)
        ctx.apply_H(Xd, Yd)
        Wd = torch.empty_like(Xd)
        ctx.chebyshev_filter(Xd, Wd, 6, 0.5 * (lo + hi), hi, lo)
        outs.append((to_np(Yd), to_np(Xd)))
    monkeypatch.delenv("SPARC_GPU_PROJ_NB", raising=False)
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_sweep_block_order_does_not_change_results(prec, monkeypatch):
    """The sweep's workgroups each write their own slab of one orbital, so
    the order in which they are dispatched (SPARC_GPU_SWEEP_GROUP orbitals'
    copies of a slab side by side: 1, the default 4, and 3, which leaves a
    short last group of the 11 orbitals) changes no result: H X and the
    filter are bitwise the same."""
    torch = require_gpu()
    s = ragged_system(n_states=11)
    v = _veff(s, 33)
    X = W.initial_orbitals(s.nd, s.n_states, 9)
    dt = torch.float64 if prec == "fp64" else torch.float32
    outs = []
    for grp in ("1", None, "3"):
        if grp:
            monkeypatch.setenv("SPARC_GPU_SWEEP_GROUP", grp)
        else:
            monkeypatch.delenv("SPARC_GPU_SWEEP_GROUP", raising=False)
        ctx = _ctx(s)
        ctx.set_veff(to_dev(torch, v))
        lo, hi = ctx.spectrum_bounds()
        Xd = to_dev(torch, X, dt)
        Yd = torch.empty_like(Xd)
        ctx.apply_H(Xd, Yd)
        Wd = torch.empty_like(Xd)
        ctx.chebyshev_filter(Xd, Wd, 6, 0.5 * (lo + hi), hi, lo)
        outs.append((to_np(Yd), to_np(Xd)))
    monkeypatch.delenv("SPARC_GPU_SWEEP_GROUP", raising=False)
    for o in outs[1:]:
        assert np.array_equal(outs[0][0], o[0])
        assert np.array_equal(outs[0][1], o[1])


def test_create_rejects_more_than_seven_supports_at_a_point():
    """4 atoms in a 4.2 x 4.5 Bohr cross-section with 3 Bohr projector
    supports: with their periodic images, 8 supports meet at some grid point
    (counted on the CPU), more than the sweep's point words hold; creation
    fails with SPARC_ERR_ARG instead of dropping a term."""
    require_gpu()
    from paper_2005_10431_amd import Context, SparcError
    s = W.tiny_system(n=(14, 16, 37), L=(4.2, 4.5, 11.1), n_atoms=4, seed=13, n_states=4)
    with pytest.raises(SparcError, match="SPARC_ERR_ARG"):
        Context(s)


def test_apply_H_wide_grid_many_halo_values():
    """200 x 14 x 13 grid: the nonlocal sweep's slab shrinks to 2 rows and
    each thread carries 6 halo values per plane."""
    torch = require_gpu()
    s = W.tiny_system(n=(200, 14, 13), L=(30.0, 4.2, 3.9), n_atoms=4, seed=9)
    log("apply_H wide grid", s.n)
    ctx = _ctx(s)
    projs = atoms.projectors(s)
    v = _veff(s, 23)
    X = W.initial_orbitals(s.nd, 5, 3)
    ctx.set_veff(to_dev(torch, v))
    Xd = to_dev(torch, X)
    Yd = torch.zeros_like(Xd)
    ctx.apply_H(Xd, Yd)
    Yref = hamiltonian.apply_H(s, v, projs, X)
    assert rel_err(to_np(Yd), Yref) <= 1e-12
