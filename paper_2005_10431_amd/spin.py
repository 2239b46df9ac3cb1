"""Throughput of the spin-polarised SCF step beside the spin-unpolarised one
(host control flow only; every step runs in the library's kernels).

Workloads: config 2 (108 atoms, 72^3, 260 states) and its spin-polarised
variant (one atom Z = 3, 431 electrons, 260 states per spin).  After the
first iteration and `--warmup` further steps, `--steps` SCF steps are timed
with HIP events; the filter sweep is timed per launch (profile id 0) and its
achieved bandwidth is the algorithmic 3 s N_d N_s bytes per column pass
divided by the mean launch time.  Optionally (--converge TOL) the spin SCF
is then run from the start to a residual below TOL.

    python -m paper_2005_10431_amd.spin --steps 10 --warmup 2
"""
from __future__ import annotations

import argparse
import json
import sys


def timed_steps(system, spin: bool, steps: int, warmup: int):
    import numpy as np
    import torch

    import workloads as W
    from ._lib import Context, make_spin_state, make_state
    nd, ns = system.nd, system.n_states
    ctx = Context(system)
    m = system.pulay_history
    rho = torch.empty((2 if spin else 1) * nd, dtype=torch.float64, device="cuda")
    eig = torch.empty((2 if spin else 1) * ns, dtype=torch.float64, device="cuda")
    occ = torch.empty_like(eig)
    hist = torch.empty((2 * m + 2) * rho.numel(), dtype=torch.float64, device="cuda") if m > 0 else None
    if spin:
        up, dn = W.initial_orbitals_spin(nd, ns, system.seed)
        Xu = torch.as_tensor(up).cuda()
        Xd = torch.as_tensor(dn).cuda()
        del up, dn
        ctx.sad_density(rho[:nd])
        z = system.spin_zeta0
        rho[nd:].copy_(rho[:nd])
        rho[:nd].mul_(0.5 * (1 + z))
        rho[nd:].mul_(0.5 * (1 - z))
        st = make_spin_state(rho, Xu, Xd, eig, occ, system.cheb_degree, system.n_first, system.mix_beta, None,
                             system.kerker_q0, m, system.pulay_period, bool(system.pulay_restart), hist)
        step = ctx.scf_step_spin
    else:
        X = torch.as_tensor(W.initial_orbitals(nd, ns, system.seed)).cuda()
        ctx.sad_density(rho)
        st = make_state(rho, X, eig, occ, system.cheb_degree, system.n_first, system.mix_beta, None,
                        system.kerker_q0, m, system.pulay_period, bool(system.pulay_restart), hist)
        step = ctx.scf_step
    step(st)
    for _ in range(warmup):
        step(st)
    ctx.profile(True)
    for k in range(20):
        ctx.profile_read(k)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    reps = [step(st) for _ in range(steps)]
    e1.record()
    torch.cuda.synchronize()
    sw_ms, sw_n = ctx.profile_read(0)
    ctx.profile(False)
    nspin = 2 if spin else 1
    # one sweep launch covers all columns of one spin block
    bytes_per_launch = 3 * 8 * nd * ns
    out = dict(
        spin=spin,
        ms_per_step=e0.elapsed_time(e1) / steps,
        t_filter_ms=float(np.median([r["t_filter_ms"] for r in reps])),
        t_rr_ms=float(np.median([r["t_rr_ms"] for r in reps])),
        t_potential_ms=float(np.median([r["t_potential_ms"] for r in reps])),
        t_density_ms=float(np.median([r["t_density_ms"] for r in reps])),
        sweep_launches=sw_n,
        sweep_ms_mean=sw_ms / sw_n if sw_n else None,
        sweep_gbs=bytes_per_launch / (sw_ms / sw_n * 1e-3) / 1e9 if sw_n else None,
        sweep_launches_per_step=sw_n / steps,
        orbital_columns_per_step=nspin * ns,
        residual=reps[-1]["residual"],
        free_per_atom=reps[-1]["free_energy"] / system.n_atoms,
    )
    ctx.close()
    torch.cuda.empty_cache()
    return out


def main(argv=None):
    import workloads as W
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--converge", type=float, default=0.0, help="also run the spin SCF to this residual (0: skip)")
    ap.add_argument("--max-iter", type=int, default=200)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    res = {}
    for name, system, spin in (("cfg2", W.config2(0), False), ("cfg2s", W.config2_spin(0), True)):
        r = timed_steps(system, spin, a.steps, a.warmup)
        res[name] = r
        log(f"{name}: {r['ms_per_step']:.2f} ms per SCF step ({r['orbital_columns_per_step']} orbital columns), "
            f"filter {r['t_filter_ms']:.2f} ms, RR {r['t_rr_ms']:.2f} ms, sweep {r['sweep_ms_mean']:.4f} ms/launch "
            f"= {r['sweep_gbs']:.0f} GB/s, {r['sweep_launches_per_step']:.0f} sweep launches per step")
    res["ratio_spin_to_unpolarised"] = res["cfg2s"]["ms_per_step"] / res["cfg2"]["ms_per_step"]
    log(f"spin / unpolarised step time: {res['ratio_spin_to_unpolarised']:.3f}")
    if a.converge > 0:
        from .driver import run_scf_spin
        s = W.config2_spin(0)
        out = run_scf_spin(s, max_iter=a.max_iter, tol=a.converge)
        h = out["history"]
        res["converge"] = dict(tol=a.converge, iterations=len(h), residual=h[-1]["residual"],
                               free_per_atom=h[-1]["free_energy"] / s.n_atoms, magnetization=h[-1]["magnetization"],
                               gpu_ms=float(sum(r["t_total_ms"] for r in h)))
        log(f"cfg2s SCF to {a.converge}: {len(h)} iterations, residual {h[-1]['residual']:.2e}, "
            f"F/atom {res['converge']['free_per_atom']:.10f}, M {h[-1]['magnetization']:.6f}")
        out["ctx"].close()
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)
    return res


if __name__ == "__main__":
    main(sys.argv[1:])
