"""Host-side SCF loop over ``sparc_gpu_scf_step`` (control flow only; each
iteration runs entirely in the library's kernels)."""
from __future__ import annotations

import numpy as np

from ._lib import SPARC_FP32, Context, make_k_state, make_spin_state, make_state


def run_scf(system, X0=None, rho0=None, prec: str = "fp64", max_iter: int = 100, tol: float = 1e-10,
            device: str = "cuda", final_fp64_rr: bool = True, ctx: Context = None, callback=None,
            n_first: int = None, degree: int = None, beta: float = None, kerker_q0: float = None,
            pulay_history: int = None, pulay_period: int = None, pulay_restart: bool = None):
    """Run the SCF iteration on the GPU.

    X0: (N_s, N_d) numpy array or tensor (random block, see
    ``workloads.initial_orbitals``; a tensor is copied, never overwritten);
    rho0: (N_d,) numpy array or float64 tensor, or None for the atomic-density
    guess.
    callback(report) is called after every iteration; a true return value
    ends the loop there (before the final FP64 Rayleigh-Ritz of the FP32 form).
    Returns a dict with the history of reports and the final device tensors."""
    import torch
    ctx = ctx or Context(system)
    nd, ns = system.nd, system.n_states
    dt = torch.float64 if prec == "fp64" else torch.float32
    if X0 is None:
        from workloads import initial_orbitals
        X0 = initial_orbitals(nd, ns, system.seed)
    if isinstance(X0, torch.Tensor):
        # a private copy: the SCF overwrites its block
        X = torch.empty((ns, nd), dtype=dt, device=device)
        X.copy_(X0)
    else:
        X = torch.as_tensor(np.asarray(X0), dtype=dt).to(device).contiguous()
    rho_in = torch.empty(nd, dtype=torch.float64, device=device)
    if rho0 is None:
        ctx.sad_density(rho_in)
    else:
        src = rho0 if isinstance(rho0, torch.Tensor) else torch.as_tensor(np.asarray(rho0), dtype=torch.float64)
        rho_in.copy_(src)
    eig = torch.empty(ns, dtype=torch.float64, device=device)
    occ = torch.empty(ns, dtype=torch.float64, device=device)
    rho_out = torch.empty(nd, dtype=torch.float64, device=device)
    m = pulay_history if pulay_history is not None else getattr(system, "pulay_history", 0)
    period = pulay_period if pulay_period is not None else getattr(system, "pulay_period", 2)
    restart = pulay_restart if pulay_restart is not None else bool(getattr(system, "pulay_restart", 0))
    hist_buf = torch.empty((2 * m + 2) * nd, dtype=torch.float64, device=device) if m > 0 else None
    st = make_state(rho_in, X, eig, occ,
                    degree if degree is not None else system.cheb_degree,
                    n_first if n_first is not None else system.n_first,
                    beta if beta is not None else system.mix_beta, rho_out,
                    kerker_q0 if kerker_q0 is not None else system.kerker_q0,
                    m, period, restart, hist_buf)
    hist = []
    for _ in range(max_iter):
        rep = ctx.scf_step(st)
        rep["eig"] = eig.detach().cpu().numpy().copy()
        hist.append(rep)
        if callback is not None and callback(rep):
            break
        if rep["residual"] < tol:
            break
    out = dict(history=hist, X=X, eig=eig, occ=occ, rho_in=rho_in, rho_out=rho_out, state=st, ctx=ctx,
               pulay_hist=hist_buf)
    if prec != "fp64" and final_fp64_rr:
        X64 = torch.empty((ns, nd), dtype=torch.float64, device=device)
        # one FP64 Rayleigh-Ritz at the (converged) input density
        rep = ctx.final_rr_fp64(st, X64)
        rep["eig"] = eig.detach().cpu().numpy().copy()
        out["final"] = rep
        out["X64"] = X64
    return out


def run_scf_spin(system, X0=None, rho0=None, prec: str = "fp64", max_iter: int = 100, tol: float = 1e-10,
                 device: str = "cuda", ctx: Context = None, callback=None, n_first: int = None,
                 degree: int = None):
    """Spin-polarised SCF on the GPU (``sparc_gpu_scf_step_spin``).

    X0: (X0_up, X0_dn) numpy arrays of shape (N_s, N_d) (default
    ``workloads.initial_orbitals_spin``); rho0: (2 N_d,) up then down, or
    None for the atomic-density guess split by ``system.spin_zeta0``.
    Mixing, preconditioner and Pulay settings come from the system.
    Each report gains "magnetization" = dV sum (rho_out_up - rho_out_dn)."""
    import torch
    ctx = ctx or Context(system)
    nd, ns = system.nd, system.n_states
    dt = torch.float64 if prec == "fp64" else torch.float32
    if X0 is None:
        from workloads import initial_orbitals_spin
        X0 = initial_orbitals_spin(nd, ns, system.seed)
    Xu = torch.as_tensor(np.asarray(X0[0]), dtype=dt).to(device).contiguous()
    Xd = torch.as_tensor(np.asarray(X0[1]), dtype=dt).to(device).contiguous()
    rho_in = torch.empty(2 * nd, dtype=torch.float64, device=device)
    if rho0 is None:
        ctx.sad_density_spin(float(getattr(system, "spin_zeta0", 0.0)), rho_in)
    else:
        src = rho0 if isinstance(rho0, torch.Tensor) else torch.as_tensor(np.asarray(rho0), dtype=torch.float64)
        rho_in.copy_(src)
    eig = torch.empty(2 * ns, dtype=torch.float64, device=device)
    occ = torch.empty(2 * ns, dtype=torch.float64, device=device)
    rho_out = torch.empty(2 * nd, dtype=torch.float64, device=device)
    m = getattr(system, "pulay_history", 0)
    hist_buf = torch.empty((2 * m + 2) * 2 * nd, dtype=torch.float64, device=device) if m > 0 else None
    st = make_spin_state(rho_in, Xu, Xd, eig, occ,
                         degree if degree is not None else system.cheb_degree,
                         n_first if n_first is not None else system.n_first,
                         system.mix_beta, rho_out, system.kerker_q0, m, getattr(system, "pulay_period", 2),
                         bool(getattr(system, "pulay_restart", 0)), hist_buf)
    hist = []
    for _ in range(max_iter):
        rep = ctx.scf_step_spin(st)
        e = eig.detach().cpu().numpy()
        rep["eig_up"], rep["eig_dn"] = e[:ns].copy(), e[ns:].copy()
        rep["magnetization"] = float(system.dV * (rho_out[:nd].sum() - rho_out[nd:].sum()).item())
        hist.append(rep)
        if callback is not None:
            callback(rep)
        if rep["residual"] < tol:
            break
    return dict(history=hist, X=(Xu, Xd), eig=eig, occ=occ, rho_in=rho_in, rho_out=rho_out, state=st, ctx=ctx,
                pulay_hist=hist_buf)


def scf_forces(system, out) -> "np.ndarray":
    """Hellmann-Feynman forces (n_atoms, 3) in Ha/Bohr after ``run_scf`` or
    ``run_scf_spin``: the electrostatic potential of the last output density
    (the density of the final orbitals), then ``sparc_gpu_forces`` with the
    final blocks and occupations."""
    import torch
    ctx = out["ctx"]
    nd = system.nd
    phi = torch.empty(nd, dtype=torch.float64, device=out["rho_out"].device)
    if isinstance(out["X"], tuple):
        ctx.potential_spin(out["rho_out"], phi)
        blocks = list(out["X"])
    else:
        ctx.potential(out["rho_out"], phi)
        blocks = [out.get("X64", out["X"])]
    F = torch.empty((system.n_atoms, 3), dtype=torch.float64, device=phi.device)
    ctx.forces(phi, blocks, out["occ"], F)
    return F.cpu().numpy()


def bloch_block(Z, dtype, device="cuda"):
    """Device block of Bloch columns for complex start orbitals Z (N_s, N_d):
    columns 2n = [Re z_n; Im z_n] and 2n + 1 = [-Im z_n; Re z_n] (the span is
    closed under z -> i z), shape (2 N_s, 2 N_d)."""
    import torch
    Z = np.asarray(Z)
    u, v = np.real(Z), np.imag(Z)
    B = np.empty((2 * Z.shape[0], 2 * Z.shape[1]))
    B[0::2, :Z.shape[1]], B[0::2, Z.shape[1]:] = u, v
    B[1::2, :Z.shape[1]], B[1::2, Z.shape[1]:] = -v, u
    return torch.as_tensor(B, dtype=dtype).to(device).contiguous()


def run_scf_k(system, kpts, kweights, Z0s=None, rho0=None, prec: str = "fp64", max_iter: int = 100,
              tol: float = 1e-10, device: str = "cuda", ctx: Context = None, callback=None, n_first: int = None,
              degree: int = None):
    """SCF over a k-point set on the GPU (``sparc_gpu_scf_step_k``).  Z0s: one
    complex (N_s, N_d) start block per k (default
    ``workloads.initial_orbitals_k``).  Each report gains "eig_k": the Ritz
    values per k with each Bloch eigenvalue once (every second entry of the
    doubled list)."""
    import torch
    ctx = ctx or Context(system)
    nd, ns = system.nd, system.n_states
    nk = len(kpts)
    dt = torch.float64 if prec == "fp64" else torch.float32
    if Z0s is None:
        from workloads import initial_orbitals_k
        Z0s = [initial_orbitals_k(nd, ns, system.seed, q) for q in range(nk)]
    blocks = [bloch_block(Z, dt, device) for Z in Z0s]
    rho_in = torch.empty(nd, dtype=torch.float64, device=device)
    if rho0 is None:
        ctx.sad_density(rho_in)
    else:
        rho_in.copy_(torch.as_tensor(np.asarray(rho0), dtype=torch.float64))
    eig = torch.empty(nk * 2 * ns, dtype=torch.float64, device=device)
    occ = torch.empty_like(eig)
    rho_out = torch.empty(nd, dtype=torch.float64, device=device)
    m = getattr(system, "pulay_history", 0)
    hist_buf = torch.empty((2 * m + 2) * nd, dtype=torch.float64, device=device) if m > 0 else None
    st = make_k_state(rho_in, blocks, kpts, kweights, eig, occ,
                      degree if degree is not None else system.cheb_degree,
                      n_first if n_first is not None else system.n_first, system.mix_beta, rho_out,
                      system.kerker_q0, m, getattr(system, "pulay_period", 2), bool(getattr(system, "pulay_restart", 0)),
                      hist_buf)
    hist = []
    for _ in range(max_iter):
        rep = ctx.scf_step_k(st)
        e = eig.detach().cpu().numpy().reshape(nk, 2 * ns)
        rep["eig_k"] = [row[0::2].copy() for row in e]
        hist.append(rep)
        if callback is not None:
            callback(rep)
        if rep["residual"] < tol:
            break
    return dict(history=hist, X=blocks, eig=eig, occ=occ, rho_in=rho_in, rho_out=rho_out, state=st, ctx=ctx,
                pulay_hist=hist_buf)
