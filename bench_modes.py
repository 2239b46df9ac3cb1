"""Measurement modes of ``bench.py`` beyond its default line (host control
flow only; every step they time runs in the library's kernels):

    python bench.py --mode mixing  ...   SCF iterations, linear vs periodic Pulay mixing
    python bench.py --mode spin    ...   spin-polarised vs unpolarised SCF step
    python bench.py --mode eigh    ...   subspace eigensolver phases
    python bench.py --mode forces  ...   Hellmann-Feynman forces after an SCF
    python bench.py --mode kpoints ...   Bloch k-point SCF step

Each mode's own options follow ``--mode NAME`` (``--help`` lists them).
"""
from __future__ import annotations

import argparse
import json
import os
import sys


# ---------------------------------------------------------------------- mixing

MIXING_DOC = """SCF iterations and time to convergence with linear (preconditioned) mixing
versus the restarted periodic Pulay mixing of Sec. 2.1 (host control flow
only; every SCF step, including the mixing, runs in the library's kernels).

For each variant the FP64 SCF runs from the seeded random block and the
atomic-density guess until the density residual is below --tol; reported:
iterations, summed GPU time of the SCF steps, the free energy per atom at
the end, the mean device time of one mixing step (profile id 19) and the
free-energy difference to the first variant.

    python bench.py --mode mixing --config cfg2 --tol 1e-7
"""

MIXING_VARIANTS = {
    # name: (pulay_history, pulay_period, pulay_restart)
    "linear": (0, 1, False),
    "pulay7p2r": (7, 2, True),
    "pulay7p2": (7, 2, False),
    "pulay7p1": (7, 1, False),
}


def mixing_run_variant(system, name, tol, max_iter, log=print):
    import torch
    import workloads as W
    from paper_2005_10431_amd._lib import Context
    from paper_2005_10431_amd.driver import run_scf
    m, period, restart = MIXING_VARIANTS[name]
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


def mixing_main(argv=None):
    import workloads as W
    ap = argparse.ArgumentParser(description=MIXING_DOC, formatter_class=argparse.RawDescriptionHelpFormatter)
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
    recs = [mixing_run_variant(system, v, a.tol, a.max_iter, log) for v in a.variants.split(",")]
    for r in recs:
        r["dF_per_atom_vs_first"] = r["free_per_atom"] - recs[0]["free_per_atom"]
    res = dict(config=a.config, tol=a.tol, variants=recs)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)
    return res


# ---------------------------------------------------------------------- spin

SPIN_DOC = """Throughput of the spin-polarised SCF step beside the spin-unpolarised one
(host control flow only; every step runs in the library's kernels).

Workloads: config 2 (108 atoms, 72^3, 260 states) and its spin-polarised
variant (one atom Z = 3, 431 electrons, 260 states per spin).  After the
first iteration and `--warmup` further steps, `--steps` SCF steps are timed
with HIP events; the filter sweep is timed per launch (profile id 0) and its
achieved bandwidth is the algorithmic 3 s N_d N_s bytes per column pass
divided by the mean launch time.  Optionally (--converge TOL) the spin SCF
is then run from the start to a residual below TOL.

    python bench.py --mode spin --steps 10 --warmup 2
"""

def spin_timed_steps(system, spin: bool, steps: int, warmup: int):
    import numpy as np
    import torch

    import workloads as W
    from paper_2005_10431_amd._lib import Context, make_spin_state, make_state
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
        ctx.sad_density_spin(system.spin_zeta0, rho)
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


def spin_main(argv=None):
    import workloads as W
    ap = argparse.ArgumentParser(description=SPIN_DOC, formatter_class=argparse.RawDescriptionHelpFormatter)
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
        r = spin_timed_steps(system, spin, a.steps, a.warmup)
        res[name] = r
        log(f"{name}: {r['ms_per_step']:.2f} ms per SCF step ({r['orbital_columns_per_step']} orbital columns), "
            f"filter {r['t_filter_ms']:.2f} ms, RR {r['t_rr_ms']:.2f} ms, sweep {r['sweep_ms_mean']:.4f} ms/launch "
            f"= {r['sweep_gbs']:.0f} GB/s, {r['sweep_launches_per_step']:.0f} sweep launches per step")
    res["ratio_spin_to_unpolarised"] = res["cfg2s"]["ms_per_step"] / res["cfg2"]["ms_per_step"]
    log(f"spin / unpolarised step time: {res['ratio_spin_to_unpolarised']:.3f}")
    if a.converge > 0:
        from paper_2005_10431_amd.driver import run_scf_spin
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


# ---------------------------------------------------------------------- eigh

EIGH_DOC = """Phase times of the subspace eigensolver (host control flow only; every step
runs in the library's kernels).

For each N, a seeded random symmetric N x N matrix is solved with the
reduction to tridiagonal form in one workgroup and with the reduction spread
over many workgroups (with its one-workgroup tail), `--reps` times each after
one untimed solve.  Reported per solve: tridiagonalisation, bisection,
inverse iteration and back-transformation (profile ids 12-15), and the
largest eigenvalue error relative to numpy.linalg.eigvalsh.

    python bench.py --mode eigh --n 260,520,1200,2000
"""

def eigh__solve(n, multi_min, tail, reps):
    import numpy as np
    import torch

    import workloads as W
    from paper_2005_10431_amd._lib import Context

    os.environ["SPARC_GPU_TRD_MULTI_MIN"] = str(multi_min)
    os.environ["SPARC_GPU_TRD_TAIL"] = str(tail)
    ctx = Context(W.tiny_system(with_nonlocal=False))
    a = np.random.default_rng(n).standard_normal((n, n))
    a = 0.5 * (a + a.T)
    A0 = torch.tensor(a.T.copy(), dtype=torch.float64, device="cuda")
    V = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    e = torch.zeros(n, dtype=torch.float64, device="cuda")
    ctx.subspace_eigh(A0.clone(), V, e)
    torch.cuda.synchronize()
    ctx.profile(True)
    for k in range(24):
        ctx.profile_read(k)
    for _ in range(reps):
        ctx.subspace_eigh(A0.clone(), V, e)
    torch.cuda.synchronize()
    out = {name: ctx.profile_read(k)[0] / reps
           for name, k in (("tridiag_ms", 12), ("bisect_ms", 13), ("invit_ms", 14), ("back_ms", 15))}
    ctx.profile(False)
    ctx.close()
    ref = np.linalg.eigvalsh(a)
    out["eig_err_rel"] = float(np.max(np.abs(e.cpu().numpy() - ref)) / np.max(np.abs(ref)))
    return out


def eigh_main(argv=None):
    ap = argparse.ArgumentParser(description=EIGH_DOC, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--n", default="260,520,1200,2000", help="comma-separated matrix sizes")
    ap.add_argument("--tail", type=int, default=256, help="rows the one-workgroup tail takes over")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    rows = []
    for n in (int(v) for v in a.n.split(",")):
        for label, mm in (("one workgroup", 1 << 30), ("many workgroups", 3)):
            r = dict(n=n, reduction=label, **eigh__solve(n, mm, a.tail, a.reps))
            rows.append(r)
            print(f"N={n:5d} {label:15s}: tridiag {r['tridiag_ms']:8.2f} ms  bisect {r['bisect_ms']:.2f}  "
                  f"inverse iteration {r['invit_ms']:.2f}  back {r['back_ms']:.2f}  "
                  f"eig err {r['eig_err_rel']:.1e}", flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(rows, f, indent=1)
    return rows


# ---------------------------------------------------------------------- forces

FORCES_DOC = """Time of the Hellmann-Feynman forces after an SCF (host control flow only;
the SCF and the forces run in the library's kernels).

Workload: config 2 (72^3 grid, 108 atoms with s + p projectors, 260
states), FP64 SCF with the workload's mixing from the seeded block to a
residual below --tol, then `--reps` evaluations of sparc_gpu_forces timed
per part with HIP events (profile ids 20: local + overlap, 21: nonlocal).
Reported with the algorithmic work of each part:
  nonlocal: every (support point, image) pair of every atom read once per
            column, 8 bytes each (the gather volume of the projection);
  local:    (point, image) pairs inside the 8 rc balls, each with one exp
            and one erf.

    python bench.py --mode forces --tol 1e-6 --reps 10
"""

def forces_ball_count(system, rmax_of_atom):
    import numpy as np
    n = 0
    h = system.h
    for I in range(system.n_atoms):
        rmax = rmax_of_atom(I)
        axes = []
        for d in range(3):
            lo = int(np.ceil((system.pos[I, d] - rmax) / h[d]))
            hi = int(np.floor((system.pos[I, d] + rmax) / h[d]))
            axes.append((np.arange(lo, hi + 1) * h[d] - system.pos[I, d]) ** 2)
        r2 = axes[0][None, None, :] + axes[1][None, :, None] + axes[2][:, None, None]
        n += int(np.count_nonzero(r2 <= rmax * rmax))
    return n


def forces_main(argv=None):
    import numpy as np
    import torch

    import workloads as W
    from paper_2005_10431_amd.driver import run_scf, scf_forces

    ap = argparse.ArgumentParser(description=FORCES_DOC, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--config", default="cfg2", choices=["cfg2", "cfg4"])
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--max-iter", type=int, default=200)
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    s = W.CONFIG_NAMES[a.config](0)
    out = run_scf(s, max_iter=a.max_iter, tol=a.tol)
    h = out["history"]
    print(f"{a.config} SCF: {len(h)} iterations, residual {h[-1]['residual']:.2e}", flush=True)
    F = scf_forces(s, out)
    ctx = out["ctx"]
    nd = s.nd
    phi = torch.empty(nd, dtype=torch.float64, device="cuda")
    ctx.potential(out["rho_out"], phi)
    Fd = torch.empty((s.n_atoms, 3), dtype=torch.float64, device="cuda")
    ctx.forces(phi, [out["X"]], out["occ"], Fd)
    torch.cuda.synchronize()
    ctx.profile(True)
    for k in range(22):
        ctx.profile_read(k)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(a.reps):
        ctx.forces(phi, [out["X"]], out["occ"], Fd)
    e1.record()
    torch.cuda.synchronize()
    loc_ms, loc_n = ctx.profile_read(20)
    nl_ms, nl_n = ctx.profile_read(21)
    ctx.profile(False)
    n_nl = forces_ball_count(s, lambda I: s.rcut_nl)
    n_loc = forces_ball_count(s, lambda I: 8.0 * s.rc_loc[I])
    nl_bytes = 8.0 * n_nl * s.n_states
    res = dict(
        config=a.config, scf_iterations=len(h), residual=h[-1]["residual"],
        forces_ms=e0.elapsed_time(e1) / a.reps,
        local_ms=loc_ms / loc_n, nonlocal_ms=nl_ms / nl_n,
        nonlocal_pairs=n_nl, local_pairs=n_loc,
        nonlocal_gather_gbs=nl_bytes / (nl_ms / nl_n * 1e-3) / 1e9,
        local_pairs_per_s=n_loc / (loc_ms / loc_n * 1e-3),
        max_abs_force=float(np.max(np.abs(F))),
        net_force=[float(v) for v in F.sum(axis=0)],
        scf_step_ms_median=float(np.median([r["t_total_ms"] for r in h[1:]])),
    )
    print(f"forces: {res['forces_ms']:.3f} ms per evaluation (local + overlap {res['local_ms']:.3f} ms, "
          f"nonlocal {res['nonlocal_ms']:.3f} ms); nonlocal gather {res['nonlocal_gather_gbs']:.0f} GB/s over "
          f"{n_nl} support pairs x {s.n_states} columns; local {res['local_pairs_per_s'] / 1e9:.2f} G pairs/s; "
          f"max |F| {res['max_abs_force']:.4e} Ha/Bohr, net force {res['net_force']}; "
          f"SCF step {res['scf_step_ms_median']:.1f} ms", flush=True)
    ctx.close()
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)
    return res


# ---------------------------------------------------------------------- kpoints

KPOINTS_DOC = """Throughput of the Bloch k-point SCF step at cfg2 scale (host control flow
only; every step runs in the library's kernels).

Workload: config 2 (72^3 grid, 108 atoms with s + p projectors, 260 states)
on a 2 x 1 x 1 Monkhorst-Pack k-point set.  Each k-point holds 520 Bloch
columns of 2 N_d rows (the 260 states and their i-multiples).  After the
first iteration and `--warmup` steps, `--steps` SCF steps are timed with HIP
events.  The Bloch filter step (profile id 22) is timed per launch.  Its
algorithmic traffic per launch is 3 x 8 x 2 N_d bytes per column (read Y_k,
read Y_{k-1}, write Y_{k+1}, both halves), which is the same count as the
Gamma sweep on a column of twice the length.

    python bench.py --mode kpoints --steps 3 --warmup 1
"""

def kpoints_main(argv=None):
    import numpy as np
    import torch

    import workloads as W
    from paper_2005_10431_amd._lib import Context, make_k_state
    from paper_2005_10431_amd.driver import bloch_block

    ap = argparse.ArgumentParser(description=KPOINTS_DOC, formatter_class=argparse.RawDescriptionHelpFormatter)
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



MODES = {"mixing": mixing_main, "spin": spin_main, "eigh": eigh_main, "forces": forces_main,
         "kpoints": kpoints_main}
