"""Parity at the full size of the largest workload (L = 34 Bohr, 120^3 grid,
500 atoms with s+p projectors, 1200 states, Chebyshev degree 24): the whole
1200-column block is processed in the launch configuration of the library,
and the oracle recomputes sampled columns one by one (every column of H X
and of the filter depends on that column alone).  FP64 to 1e-12 (H X) and
1e-11 (filter) relative; FP32 H X to 2e-6 and the FP32 filter to
2 m 2e-6 (each sweep at most one FP32 H X error, adding linearly)."""
import numpy as np
import pytest

import workloads as W
from oracle import atoms, chefsi, hamiltonian

from gpu_helpers import log, rel_err, require_gpu, to_dev, to_np

pytestmark = pytest.mark.gpu


def _block(torch, s, seed, keep):
    """The seeded FP64 start block, streamed to the device in row chunks; the
    rows listed in `keep` are also returned on the host."""
    X = torch.empty((s.n_states, s.nd), dtype=torch.float64, device="cuda")
    rows_kept = {}
    for r0, rows in W.initial_orbitals_rows(s.nd, s.n_states, seed, rows=64):
        X[r0:r0 + rows.shape[0]] = torch.as_tensor(rows).cuda()
        for j in keep:
            if r0 <= j < r0 + rows.shape[0]:
                rows_kept[j] = rows[j - r0].copy()
    return X, rows_kept


def test_cfg4_full_block_apply_and_filter():
    torch = require_gpu()
    from paper_2005_10431_amd import Context
    s = W.config4(0)
    log("cfg4: 120^3 grid, 500 atoms, 1200 states")
    ctx = Context(s)
    projs = atoms.projectors(s)
    v = np.random.default_rng(31).uniform(-1.0, 1.0, s.nd)
    ctx.set_veff(to_dev(torch, v))
    cols = (0, 613, 1199)
    X, ref_rows = _block(torch, s, 2, cols)
    X32 = X.to(torch.float32)
    Y = torch.empty_like(X)
    ctx.apply_H(X, Y)
    torch.cuda.synchronize()
    for j in cols:
        yref = hamiltonian.apply_H(s, v, projs, ref_rows[j][None])[0]
        err = rel_err(to_np(Y[j]), yref)
        log(f"  H X column {j}: rel err {err:.2e}")
        assert err <= 1e-12
    del Y

    lo, hi = hamiltonian.spectrum_bounds(s, v, projs)
    a, b, a0 = lo + 0.05 * (hi - lo), hi, lo
    Wk = torch.empty_like(X)
    ctx.chebyshev_filter(X, Wk, s.cheb_degree, a, b, a0)
    torch.cuda.synchronize()
    del Wk
    j = 613
    yref = chefsi.chebyshev_filter(s, v, projs, ref_rows[j][None], s.cheb_degree, a, b, a0)[0]
    err = rel_err(to_np(X[j]), yref)
    log(f"  filter (degree {s.cheb_degree}) column {j}: rel err {err:.2e}")
    assert err <= 1e-11
    del X
    torch.cuda.empty_cache()

    Y32 = torch.empty_like(X32)
    ctx.apply_H(X32, Y32)
    torch.cuda.synchronize()
    for j in (0, 1199):
        yref = hamiltonian.apply_H(s, v, projs, ref_rows[j].astype(np.float32).astype(np.float64)[None])[0]
        err = rel_err(to_np(Y32[j]).astype(np.float64), yref)
        log(f"  FP32 H X column {j}: rel err {err:.2e}")
        assert err <= 2e-6


def test_cfg4_full_block_fp32_filter():
    """Degree-24 FP32 filter with projectors over the full 1200-column block;
    the oracle filters one FP32-rounded column alone in FP64."""
    torch = require_gpu()
    from paper_2005_10431_amd import Context
    s = W.config4(0)
    log("cfg4 FP32 filter: 120^3 grid, 500 atoms, 1200 states")
    ctx = Context(s)
    projs = atoms.projectors(s)
    v = np.random.default_rng(32).uniform(-1.0, 1.0, s.nd)
    ctx.set_veff(to_dev(torch, v))
    j = 977
    X, ref_rows = _block(torch, s, 4, (j,))
    X32 = X.to(torch.float32)
    del X
    torch.cuda.empty_cache()
    lo, hi = hamiltonian.spectrum_bounds(s, v, projs)
    a, b, a0 = lo + 0.05 * (hi - lo), hi, lo
    Wk = torch.empty_like(X32)
    ctx.chebyshev_filter(X32, Wk, s.cheb_degree, a, b, a0)
    torch.cuda.synchronize()
    x32 = ref_rows[j].astype(np.float32).astype(np.float64)
    yref = chefsi.chebyshev_filter(s, v, projs, x32[None], s.cheb_degree, a, b, a0)[0]
    err = rel_err(to_np(X32[j]).astype(np.float64), yref)
    bar = 2.0 * s.cheb_degree * 2e-6
    log(f"  FP32 filter (degree {s.cheb_degree}) column {j}: rel err {err:.2e} (bar {bar:.1e})")
    assert err <= bar
