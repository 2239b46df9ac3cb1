"""Learned warm start of the SCF: data generation, training and evaluation
(host control flow only; features, network, gradient, Adam and every SCF
step run in the library's kernels).

Workload: the config-1 cell and physics on a 72^3 grid, geometries displaced
from the config-1 atoms by N(0, 0.15 Bohr) (``workloads.config5_snapshot``):
snapshots 0..199 train, 200..249 test.  Targets are the converged
self-consistent densities of each snapshot (FP64 SCF from the atomic-density
guess).  The figure of merit is the number of SCF iterations (and the GPU
time) until the free energy stays within 1e-6 Ha/atom of the converged
value, starting from the network's density versus the atomic-density guess.

    python -m paper_2005_10431_amd.warmstart --train 200 --test 50 --epochs 40
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def converge(system, rho0=None, tol=1e-10, max_iter=300, ctx=None, n_first=None, degree=None):
    """FP64 GPU SCF; returns (history, rho_fixed_point (device), ctx)."""
    from .driver import run_scf
    import workloads as W
    X0 = W.initial_orbitals(system.nd, system.n_states, system.seed)
    out = run_scf(system, X0, rho0=rho0, prec="fp64", max_iter=max_iter, tol=tol, ctx=ctx, n_first=n_first,
                  degree=degree)
    return out["history"], out["rho_out"], out["ctx"]


def iterations_to(hist, f_ref, n_atoms, eps=1e-6):
    """First iteration (1-based) after which |F/atom - F_ref/atom| <= eps for
    the rest of the run."""
    f = np.array([h["free_energy"] for h in hist]) / n_atoms
    ok = np.abs(f - f_ref / n_atoms) <= eps
    k = len(ok)
    while k > 0 and ok[k - 1]:
        k -= 1
    return k + 1 if k < len(ok) else None


def time_to(hist, k):
    return float(sum(h["t_total_ms"] for h in hist[:k])) if k else None


def make_dataset(seeds, n=72, log=print):
    import torch
    import workloads as W
    from ._lib import Context
    data = []
    for i, s in enumerate(seeds):
        sysm = W.config5_snapshot(s, n=n)
        hist, rho, ctx = converge(sysm, tol=1e-9)
        feat = torch.empty((3, sysm.nd), dtype=torch.float32, device="cuda")
        ctx.features(feat)
        torch.cuda.synchronize()
        ctx.close()
        data.append(dict(seed=s, system=sysm, feat=feat, target=rho.clone(), iters=len(hist),
                         f_ref=hist[-1]["free_energy"], hist=hist))
        if i % 10 == 0 or i == len(seeds) - 1:
            log(f"  snapshot {s}: {len(hist)} SCF iterations, F/atom {hist[-1]['free_energy'] / sysm.n_atoms:.10f}")
    return data


def train(data, epochs=20, lr=1e-3, seed=0, log=print):
    import torch
    import workloads as W
    from ._lib import CNN_NPARAMS, Context
    # the network and its gradient depend on the grid, N_e and dV only
    ctx = Context(data[0]["system"])
    nd = data[0]["system"].nd
    w = torch.as_tensor(W.cnn_initial_weights(seed)).cuda()
    m = torch.zeros(CNN_NPARAMS, dtype=torch.float32, device="cuda")
    v = torch.zeros_like(m)
    grad = torch.empty_like(m)
    act = torch.empty((33, nd), dtype=torch.float32, device="cuda")
    rho = torch.empty(nd, dtype=torch.float64, device="cuda")
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    rng = np.random.default_rng([seed, 17])
    t = 0
    curve = []
    t0 = time.perf_counter()
    for ep in range(epochs):
        order = rng.permutation(len(data))
        tot = 0.0
        for j in order:
            d = data[j]
            ctx.cnn_forward(w, d["feat"], act, rho)
            ctx.cnn_backward(w, d["feat"], act, rho, d["target"], grad, loss)
            t += 1
            ctx.adam_step(w, grad, m, v, t, lr=lr)
            tot += float(loss.item())
        curve.append(tot / len(data))
        log(f"  epoch {ep}: mean loss {curve[-1]:.4e}")
    torch.cuda.synchronize()
    ctx.close()
    return w, curve, time.perf_counter() - t0


def evaluate(w, data, max_l1=0.5, eps=1e-6, log=print, n_first=None, degree=None):
    """SCF from the network's density against SCF from the atomic guess, both
    with `n_first` filter passes in the first iteration and Chebyshev degree
    `degree` (the system's values when None)."""
    import torch
    from ._lib import Context
    rows = []
    for d in data:
        s = d["system"]
        if (n_first is not None and n_first != s.n_first) or (degree is not None and degree != s.cheb_degree):
            hist_sad, _, ctx0 = converge(s, tol=1e-9, n_first=n_first, degree=degree)
            ctx0.close()
        else:
            hist_sad = d["hist"]
        ctx = Context(s)
        rho0 = torch.empty(s.nd, dtype=torch.float64, device="cuda")
        used = ctx.warm_start(w, rho0, max_l1=max_l1)
        # distances of the starting densities to the converged one
        sad = torch.empty_like(rho0)
        ctx.sad_density(sad)
        pred = torch.empty_like(rho0)
        ctx.warm_start(w, pred, max_l1=float("inf"))
        l1_sad = float((sad - d["target"]).abs().sum()) * s.dV / s.n_electrons
        l1_cnn = float((pred - d["target"]).abs().sum()) * s.dV / s.n_electrons
        hist_cnn, _, _ = converge(s, rho0=rho0, tol=1e-9, ctx=ctx, n_first=n_first, degree=degree)
        torch.cuda.synchronize()
        ctx.close()
        k_sad = iterations_to(hist_sad, d["f_ref"], s.n_atoms, eps)
        k_cnn = iterations_to(hist_cnn, d["f_ref"], s.n_atoms, eps)
        rows.append(dict(seed=d["seed"], used_cnn=used, iters_sad=k_sad, iters_cnn=k_cnn,
                         ms_sad=time_to(hist_sad, k_sad), ms_cnn=time_to(hist_cnn, k_cnn),
                         f_diff=abs(hist_cnn[-1]["free_energy"] - d["f_ref"]) / s.n_atoms,
                         l1_sad=l1_sad, l1_cnn=l1_cnn))
        log(f"  test snapshot {d['seed']}: SAD {k_sad} its, warm start {k_cnn} its (CNN used: {used}); "
            f"L1 to converged density: SAD {l1_sad:.4f}, CNN {l1_cnn:.4f}")
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=200)
    ap.add_argument("--test", type=int, default=50)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--grid", type=int, default=72)
    ap.add_argument("--eval-first", type=int, nargs="+", default=[None],
                    help="first-iteration filter passes of the evaluation runs (default: the system's)")
    ap.add_argument("--eval-degree", type=int, default=None,
                    help="Chebyshev degree of the evaluation runs (default: the system's)")
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    t0 = time.perf_counter()
    log(f"training data: snapshots 0..{args.train - 1}")
    train_set = make_dataset(range(args.train), n=args.grid, log=log)
    log(f"test data: snapshots 200..{200 + args.test - 1}")
    test_set = make_dataset(range(200, 200 + args.test), n=args.grid, log=log)
    w, curve, t_train = train(train_set, epochs=args.epochs, lr=args.lr, log=log)
    evals = []
    for nf in args.eval_first:
        log(f"evaluation with {nf if nf is not None else 'default'} first-iteration passes")
        rows = evaluate(w, test_set, log=log, n_first=nf, degree=args.eval_degree)
        k_sad = [r["iters_sad"] for r in rows if r["iters_sad"]]
        k_cnn = [r["iters_cnn"] for r in rows if r["iters_cnn"]]
        ms_sad = [r["ms_sad"] for r in rows if r["ms_sad"]]
        ms_cnn = [r["ms_cnn"] for r in rows if r["ms_cnn"]]
        ev = dict(
            n_first=nf if nf is not None else test_set[0]["system"].n_first,
            degree=args.eval_degree if args.eval_degree is not None else test_set[0]["system"].cheb_degree,
            mean_iters_sad=float(np.mean(k_sad)), mean_iters_cnn=float(np.mean(k_cnn)),
            mean_ms_sad=float(np.mean(ms_sad)), mean_ms_cnn=float(np.mean(ms_cnn)),
            cnn_used=int(sum(r["used_cnn"] for r in rows)),
            mean_l1_sad=float(np.mean([r["l1_sad"] for r in rows])),
            mean_l1_cnn=float(np.mean([r["l1_cnn"] for r in rows])),
            max_f_diff=float(max(r["f_diff"] for r in rows)), rows=rows)
        log(json.dumps({k: v for k, v in ev.items() if k != "rows"}))
        evals.append(ev)
    summary = dict(
        workload=f"cfg1 cell and physics on a {args.grid}^3 grid, snapshots N(0, 0.15 Bohr)",
        n_train=args.train, n_test=args.test, epochs=args.epochs, lr=args.lr,
        loss_curve=curve, train_seconds=t_train, evaluations=evals,
        total_seconds=time.perf_counter() - t0,
    )
    if args.out:
        with open(args.out, "w") as f:
            json.dump(summary, f, indent=1)
    return summary


if __name__ == "__main__":
    sys.exit(0 if main() else 1)
