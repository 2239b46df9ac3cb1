"""Throughput of the Bloch k-point SCF step at cfg2 scale (host control flow
only; every step runs in the library's kernels).

Workload: config 2 (72^3 grid, 108 atoms with s + p projectors, 260 states)
on a 2 x 1 x 1 Monkhorst-Pack k-point set.  Each k-point holds 520 Bloch
columns of 2 N_d rows (the 260 states and their i-multiples).  After the
first iteration and `--warmup` steps, `--steps` SCF steps are timed with HIP
events.  The Bloch filter step (profile id 22) is timed per launch.  Its
algorithmic traffic per launch is 3 x 8 x 2 N_d bytes per column (read Y_k,
read Y_{k-1}, write Y_{k+1}, both halves), which is the same count as the
Gamma sweep on a column of twice the length.

    python -m paper_2005_10431_amd.kpoint_timing --steps 3 --warmup 1
"""
from __future__ import annotations

import argparse
import json
import sys


def main(argv=None):
    import numpy as np
    import torch

    import workloads as W
    from ._lib import Context, make_k_state
    from .driver import bloch_block

    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--grid", default="2,1,1")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    s = W.config2(0)
    nd, ns = s.nd, s.n_states
    kpts, wk = W.monkhorst_pack(s.L, tuple(int(v) for v in a.grid.split(",")))
    nk = len(kpts)
    ctx = Context(s)
    blocks = [bloch_block(W.initial_orbitals_k(nd, ns, s.seed, q), torch.float64) for q in range(nk)]
    rho = torch.empty(nd, dtype=torch.float64, device="cuda")
    ctx.sad_density(rho)
    eig = torch.empty(nk * 2 * ns, dtype=torch.float64, device="cuda")
    occ = torch.empty_like(eig)
    m = s.pulay_history
    hist = torch.empty((2 * m + 2) * nd, dtype=torch.float64, device="cuda") if m > 0 else None
    st = make_k_state(rho, blocks, kpts, wk, eig, occ, s.cheb_degree, s.n_first, s.mix_beta, None, s.kerker_q0, m,
                      s.pulay_period, bool(s.pulay_restart), hist)
    first = ctx.scf_step_k(st)
    print(f"first iteration {first['t_total_ms']:.0f} ms", flush=True)
    for _ in range(a.warmup):
        ctx.scf_step_k(st)
    ctx.profile(True)
    for k in range(24):
        ctx.profile_read(k)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    reps = [ctx.scf_step_k(st) for _ in range(a.steps)]
    e1.record()
    torch.cuda.synchronize()
    sw_ms, sw_n = ctx.profile_read(22)
    pj_ms, pj_n = ctx.profile_read(23)
    ctx.profile(False)
    ncol = 2 * ns
    bytes_launch = 3 * 8 * 2 * nd * ncol
    res = dict(
        workload=f"cfg2 (72^3, 108 atoms, 260 states), {nk} k-points ({a.grid} Monkhorst-Pack), FP64",
        ms_per_step=e0.elapsed_time(e1) / a.steps,
        t_filter_ms=float(np.median([r["t_filter_ms"] for r in reps])),
        t_rr_ms=float(np.median([r["t_rr_ms"] for r in reps])),
        bloch_launches=sw_n, bloch_ms_mean=sw_ms / sw_n,
        bloch_gbs=bytes_launch / (sw_ms / sw_n * 1e-3) / 1e9,
        bloch_frac=bytes_launch / (sw_ms / sw_n * 1e-3) / 8e12,
        proj_ms_mean=pj_ms / pj_n,
        residual=reps[-1]["residual"],
        free_per_atom=reps[-1]["free_energy"] / s.n_atoms,
        first_iteration_ms=first["t_total_ms"],
    )
    print(f"k-point SCF step: {res['ms_per_step']:.1f} ms ({nk} k-points, {ncol} Bloch columns each): filter "
          f"{res['t_filter_ms']:.1f} ms, RR {res['t_rr_ms']:.1f} ms; Bloch step {res['bloch_ms_mean']:.3f} ms/launch "
          f"= {res['bloch_gbs']:.0f} GB/s ({100 * res['bloch_frac']:.1f} % of 8 TB/s); projection "
          f"{res['proj_ms_mean']:.3f} ms/launch", flush=True)
    ctx.close()
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)
    return res


if __name__ == "__main__":
    main(sys.argv[1:])
