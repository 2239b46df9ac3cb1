"""SCF iterations and time to convergence with linear (preconditioned) mixing
versus the restarted periodic Pulay mixing of Sec. 2.1 (host control flow
only; every SCF step, including the mixing, runs in the library's kernels).

For each variant the FP64 SCF runs from the seeded random block and the
atomic-density guess until the density residual is below --tol; reported:
iterations, summed GPU time of the SCF steps, the free energy per atom at
the end, the mean device time of one mixing step (profile id 19) and the
free-energy difference to the first variant.

    python -m paper_2005_10431_amd.mixing --config cfg2 --tol 1e-7
"""
from __future__ import annotations

import argparse
import json
import sys

VARIANTS = {
    # name: (pulay_history, pulay_period, pulay_restart)
    "linear": (0, 1, False),
    "pulay7p2r": (7, 2, True),
    "pulay7p2": (7, 2, False),
    "pulay7p1": (7, 1, False),
}


def run_variant(system, name, tol, max_iter, log=print):
    import torch
    import workloads as W
    from ._lib import Context
    from .driver import run_scf
    m, period, restart = VARIANTS[name]
    ctx = Context(system)
    ctx.profile(True)
    X0 = W.initial_orbitals(system.nd, system.n_states, system.seed)
    out = run_scf(system, X0, prec="fp64", max_iter=max_iter, tol=tol, ctx=ctx, pulay_history=m,
                  pulay_period=period, pulay_restart=restart)
    mix_ms, mix_n = ctx.profile_read(19)
    hist = out["history"]
    torch.cuda.synchronize()
    rec = dict(variant=name, pulay_history=m, pulay_period=period, pulay_restart=restart,
               kerker_q0=system.kerker_q0, beta=system.mix_beta, iterations=len(hist),
               converged=bool(hist[-1]["residual"] < tol), residual=hist[-1]["residual"],
               scf_gpu_ms=float(sum(h["t_total_ms"] for h in hist)),
               free_per_atom=hist[-1]["free_energy"] / system.n_atoms,
               mix_ms_mean=(mix_ms / mix_n) if mix_n else None, mix_launch_groups=mix_n,
               residuals=[h["residual"] for h in hist])
    res = rec["residuals"]
    rec["iterations_to"] = {f"{t:.0e}": next((k + 1 for k, r in enumerate(res) if r < t), None)
                            for t in (1e-3, 1e-4, 1e-5, 1e-6, 1e-7)}
    ctx.close()
    del out
    torch.cuda.empty_cache()
    log(f"{name}: {rec['iterations']} iterations, converged {rec['converged']}, "
        f"SCF GPU time {rec['scf_gpu_ms']:.0f} ms, F/atom {rec['free_per_atom']:.12f}, "
        f"mix step {rec['mix_ms_mean'] if rec['mix_ms_mean'] is None else round(rec['mix_ms_mean'], 4)} ms, "
        f"iterations to residual {rec['iterations_to']}")
    return rec


def main(argv=None):
    import workloads as W
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--config", default="cfg2", choices=sorted(W.CONFIG_NAMES))
    ap.add_argument("--tol", type=float, default=1e-7)
    ap.add_argument("--max-iter", type=int, default=200)
    ap.add_argument("--variants", default="linear,pulay7p2r,pulay7p2")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    system = W.CONFIG_NAMES[a.config](0)

    def log(msg):
        print(msg, flush=True)

    log(f"{a.config}: N_d = {system.nd}, N_s = {system.n_states}, tol {a.tol}")
    recs = [run_variant(system, v, a.tol, a.max_iter, log) for v in a.variants.split(",")]
    for r in recs:
        r["dF_per_atom_vs_first"] = r["free_per_atom"] - recs[0]["free_per_atom"]
    res = dict(config=a.config, tol=a.tol, variants=recs)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)
    return res


if __name__ == "__main__":
    main(sys.argv[1:])
