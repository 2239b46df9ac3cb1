"""The allocation-free filter entry point (sparc_gpu_chebyshev_filter_noalloc)
against the regular one on the same inputs: two calls in a row on one
context, the second on a smaller block.  Both compute the same sums in the
same order (the partials' z ranges come from the whole block however its
columns are grouped), so the bar is bitwise equality; the FP64 filter bar of
the parity tests (1e-11 relative) would also do.  On the full-size workload
the partials of 600 columns exceed the fixed 32 MiB array, so the columns
run in several groups, and device memory does not shrink during the
allocation-free call while the regular call's first use allocates its
partials."""
import numpy as np
import pytest

import workloads as W

from gpu_helpers import log, ragged_system, require_gpu, to_dev

pytestmark = pytest.mark.gpu


def _bounds(ctx):
    lo, hi = ctx.spectrum_bounds()
    return lo + 0.3 * (hi - lo), hi, lo


def _both(torch, ctx, X0, degree, a, b, a0, first_noalloc=False):
    """Filter copies of X0 with both entry points; returns (regular, noalloc)."""
    Xr, Xn = X0.clone(), X0.clone()
    Wr, Wn = torch.empty_like(X0), torch.empty_like(X0)
    torch.cuda.synchronize()
    calls = [("noalloc", Xn, Wn), ("regular", Xr, Wr)] if first_noalloc else [("regular", Xr, Wr), ("noalloc", Xn, Wn)]
    for name, X, Wk in calls:
        if name == "noalloc":
            ctx.chebyshev_filter_noalloc(X, Wk, degree, a, b, a0)
        else:
            ctx.chebyshev_filter(X, Wk, degree, a, b, a0)
    torch.cuda.synchronize()
    return Xr, Xn


def _same(torch, Xr, Xn, what):
    diff = float((Xr.double() - Xn.double()).abs().max())
    scale = float(Xr.double().abs().max())
    log(f"  {what}: max |noalloc - regular| = {diff:.3e} (scale {scale:.3e})")
    assert torch.equal(Xr, Xn)


@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_noalloc_filter_matches_filter_small(dtype):
    torch = require_gpu()
    from paper_2005_10431_amd import Context
    s = ragged_system(n_states=6)
    ctx = Context(s)
    ctx.set_veff(to_dev(torch, np.random.default_rng(41).uniform(-0.5, 0.5, s.nd)))
    a, b, a0 = _bounds(ctx)
    dt = getattr(torch, dtype)
    g = torch.Generator(device="cuda").manual_seed(5)
    for ncol, degree in ((6, 9), (3, 4)):
        log(f"small ragged system, {dtype}, {ncol} columns, degree {degree}")
        X0 = torch.rand((ncol, s.nd), generator=g, device="cuda", dtype=torch.float64).to(dt) - 0.5
        Xr, Xn = _both(torch, ctx, X0, degree, a, b, a0)
        _same(torch, Xr, Xn, f"{ncol} columns")


def test_noalloc_filter_matches_filter_full_size_in_column_groups():
    torch = require_gpu()
    from paper_2005_10431_amd import Context
    s = W.config4(0)
    log("120^3 grid, 500 atoms: noalloc filter vs filter, 600 then 150 columns, degree 24")
    ctx = Context(s)
    ctx.set_veff(to_dev(torch, np.random.default_rng(42).uniform(-1.0, 1.0, s.nd)))
    a, b, a0 = _bounds(ctx)
    g = torch.Generator(device="cuda").manual_seed(6)
    X0 = torch.rand((600, s.nd), generator=g, device="cuda", dtype=torch.float64) - 0.5
    # first call on a fresh context: the allocation-free entry point before
    # the regular one has allocated anything
    Xr, Xn = X0.clone(), X0.clone()
    Wr, Wn = torch.empty_like(X0), torch.empty_like(X0)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    ctx.chebyshev_filter_noalloc(Xn, Wn, s.cheb_degree, a, b, a0)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    ctx.chebyshev_filter(Xr, Wr, s.cheb_degree, a, b, a0)
    torch.cuda.synchronize()
    free2 = torch.cuda.mem_get_info()[0]
    log(f"  device memory taken: noalloc call {free0 - free1} bytes, regular call {free1 - free2} bytes")
    assert free0 - free1 < 4 << 20
    assert free1 - free2 >= 32 << 20   # the regular call's partials exceed the fixed array
    _same(torch, Xr, Xn, "600 columns")
    del Xr, Xn, Wr, Wn
    X1 = X0[:150].clone()
    del X0
    Xr, Xn = _both(torch, ctx, X1, s.cheb_degree, a, b, a0, first_noalloc=True)
    _same(torch, Xr, Xn, "150 columns")
