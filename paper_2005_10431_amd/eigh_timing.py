"""Phase times of the subspace eigensolver (host control flow only; every step
runs in the library's kernels).

For each N, a seeded random symmetric N x N matrix is solved with the
reduction to tridiagonal form in one workgroup and with the reduction spread
over many workgroups (with its one-workgroup tail), `--reps` times each after
one untimed solve.  Reported per solve: tridiagonalisation, bisection,
inverse iteration and back-transformation (profile ids 12-15), and the
largest eigenvalue error relative to numpy.linalg.eigvalsh.

    python -m paper_2005_10431_amd.eigh_timing --n 260,520,1200,2000
"""
from __future__ import annotations

import argparse
import json
import os
import sys


def _solve(n, multi_min, tail, reps):
    import numpy as np
    import torch

    import workloads as W
    from ._lib import Context

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


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--n", default="260,520,1200,2000", help="comma-separated matrix sizes")
    ap.add_argument("--tail", type=int, default=256, help="rows the one-workgroup tail takes over")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    rows = []
    for n in (int(v) for v in a.n.split(",")):
        for label, mm in (("one workgroup", 1 << 30), ("many workgroups", 3)):
            r = dict(n=n, reduction=label, **_solve(n, mm, a.tail, a.reps))
            rows.append(r)
            print(f"N={n:5d} {label:15s}: tridiag {r['tridiag_ms']:8.2f} ms  bisect {r['bisect_ms']:.2f}  "
                  f"inverse iteration {r['invit_ms']:.2f}  back {r['back_ms']:.2f}  "
                  f"eig err {r['eig_err_rel']:.1e}", flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(rows, f, indent=1)
    return rows


if __name__ == "__main__":
    main(sys.argv[1:])
