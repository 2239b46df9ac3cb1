"""Seeded synthetic workloads shared by the oracle, the GPU binding, the tests
and the benchmark.

This module only draws inputs: atom positions, per-atom constants, projector
energies and the random starting block of orbitals.  It contains none of the
method's arithmetic (no stencil, no potential, no eigensolver), so that the CPU
oracle and the HIP path can both consume the same inputs without sharing any
numerics.

The physical systems are stand-ins for the 100-500 atom workloads of the
paper's performance discussion (Sec. 4): model atoms with a Gaussian-smeared
local pseudopotential V(r) = -Z erf(r/rc)/r and, optionally, one s and three p
Kleinman-Bylander projectors with Gaussian radial parts.  The paper's own
systems need pseudopotential files and structures that are not available, so
they are not reproduced.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Optional, Tuple

import numpy as np

__all__ = [
    "System",
    "random_positions",
    "fcc_jittered",
    "config1",
    "config2",
    "config3",
    "config4",
    "config5_snapshot",
    "config1_spin",
    "config2_spin",
    "initial_orbitals_spin",
    "initial_orbitals_k",
    "monkhorst_pack",
    "tiny_system",
    "initial_orbitals",
    "CONFIG_NAMES",
]


@dataclass
class System:
    """Everything that defines one Kohn-Sham problem on a periodic grid.

    Grid: ``n = (Nx, Ny, Nz)`` points on an orthorhombic cell of lengths
    ``L = (Lx, Ly, Lz)`` Bohr; point (ix, iy, iz) sits at (ix*hx, iy*hy, iz*hz)
    and has flat index ``ix + Nx*(iy + Ny*iz)``.
    """

    name: str
    n: Tuple[int, int, int]
    L: Tuple[float, float, float]
    pos: np.ndarray                  # (n_atoms, 3) Bohr, inside [0, L)
    Z: np.ndarray                    # (n_atoms,) valence charge
    rc_loc: np.ndarray               # (n_atoms,) Gaussian width of the local part
    n_states: int
    n_electrons: float
    kT: float = 0.01                 # Hartree, Fermi-Dirac smearing
    fd_half_order: int = 6           # 12th-order centred differences
    nl_lmax: int = -1                # -1: no nonlocal part, 1: s + p projectors
    gamma: Optional[np.ndarray] = None   # (n_atoms, nl_lmax+1) Hartree
    rc_nl: float = 1.2
    rcut_nl: float = 3.6
    rho_floor: float = 1e-14
    sad_width: float = 1.0           # Bohr, width of the atomic model densities
    cheb_degree: int = 12
    mix_beta: float = 0.3
    kerker_q0: float = 0.0     # 0: plain linear mixing
    pulay_history: int = 0     # 0: no Pulay extrapolation (linear mixing only)
    pulay_period: int = 2      # Pulay extrapolation every pulay_period-th iteration
    pulay_restart: int = 0     # 1: discard the history after a Pulay step on a full history
    n_first: int = 4                 # filter passes in the first SCF iteration
    spin: int = 1                    # 1: spin-unpolarised, 2: spin-polarised (n_states per spin)
    spin_zeta0: float = 0.0          # starting polarisation of the split atomic-density guess
    seed: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def n_atoms(self) -> int:
        return int(self.pos.shape[0])

    @property
    def nd(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    @property
    def h(self) -> Tuple[float, float, float]:
        return tuple(self.L[d] / self.n[d] for d in range(3))

    @property
    def dV(self) -> float:
        hx, hy, hz = self.h
        return hx * hy * hz

    def with_grid(self, n: Tuple[int, int, int]) -> "System":
        return replace(self, n=tuple(int(v) for v in n))


def _min_image(d: np.ndarray, L: np.ndarray) -> np.ndarray:
    return d - L * np.round(d / L)


def random_positions(L, n_atoms: int, min_sep: float, rng: np.random.Generator,
                     max_tries: int = 100000) -> np.ndarray:
    """Sequential rejection sampling of uniform positions in the periodic
    cell, keeping every minimum-image pair distance >= ``min_sep``."""
    L = np.asarray(L, dtype=np.float64)
    pos = []
    tries = 0
    while len(pos) < n_atoms:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place atoms at the requested separation")
        p = rng.uniform(0.0, 1.0, 3) * L
        ok = True
        for q in pos:
            d = _min_image(p - q, L)
            if float(np.sqrt(np.dot(d, d))) < min_sep:
                ok = False
                break
        if ok:
            pos.append(p)
    return np.array(pos, dtype=np.float64)


def fcc_jittered(L: float, ncell: int, sigma: float, rng: np.random.Generator) -> np.ndarray:
    """Face-centred cubic lattice of ``ncell**3`` conventional cells (4 atoms
    each) filling a cube of side ``L``, every coordinate displaced by
    N(0, sigma) and wrapped back into the cell."""
    a = L / ncell
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]], dtype=np.float64)
    # offset the lattice by a quarter cell so that atoms do not sit on grid planes
    off = np.array([0.25, 0.25, 0.25])
    pts = []
    for k in range(ncell):
        for j in range(ncell):
            for i in range(ncell):
                for b in basis:
                    pts.append((np.array([i, j, k], dtype=np.float64) + b + off) * a)
    pos = np.array(pts)
    pos = pos + rng.normal(0.0, sigma, pos.shape)
    return np.mod(pos, L)


def _gamma(n_atoms: int, lmax: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng([seed, 7])
    return rng.uniform(-1.0, 1.0, (n_atoms, lmax + 1))


def config1(seed: int = 0, n: int = 24) -> System:
    """L = 8 Bohr cube, 24^3 grid, 8 atoms (Z = 2, rc = 0.8) at uniform random
    positions with minimum separation 2 Bohr, no nonlocal part, 12 states for
    16 electrons, kT = 0.01 Ha, Chebyshev degree 12, linear mixing 0.3."""
    rng = np.random.default_rng(seed)
    L = 8.0
    pos = random_positions((L, L, L), 8, 2.0, rng)
    na = pos.shape[0]
    return System(
        name="cfg1", n=(n, n, n), L=(L, L, L), pos=pos,
        Z=np.full(na, 2.0), rc_loc=np.full(na, 0.8),
        n_states=12, n_electrons=16.0, kT=0.01, cheb_degree=12, mix_beta=0.3,
        seed=seed,
    )


def config2(seed: int = 0) -> System:
    """L = 20 Bohr cube, 72^3 grid, 108 atoms (FCC 3x3x3 conventional cells,
    jitter N(0, 0.1)), Z = 4, rc_loc = 1.0, s+p projectors with rc = 1.2 and
    energies U[-1, 1] Ha, 260 states for 432 electrons, degree 20.  Mixing:
    restarted periodic Pulay (history 7, period 2) with beta = 0.3 and the
    Kerker-type residual preconditioner q0 = 1 / Bohr (plain linear mixing
    sloshes at this cell size)."""
    rng = np.random.default_rng(seed)
    L = 20.0
    pos = fcc_jittered(L, 3, 0.1, rng)
    na = pos.shape[0]
    return System(
        name="cfg2", n=(72, 72, 72), L=(L, L, L), pos=pos,
        Z=np.full(na, 4.0), rc_loc=np.full(na, 1.0),
        n_states=260, n_electrons=432.0, kT=0.01, cheb_degree=20, mix_beta=0.3, kerker_q0=1.0,
        pulay_history=7, pulay_period=2, pulay_restart=1,
        nl_lmax=1, gamma=_gamma(na, 1, seed), rc_nl=1.2, rcut_nl=3.6, seed=seed,
    )


def config3(seed: int = 0) -> System:
    """The FP32-filter form of config 1 (same system; precision is chosen by
    the caller)."""
    s = config1(seed)
    s.name = "cfg3"
    return s


def config4(seed: int = 0) -> System:
    """L = 34 Bohr cube, 120^3 grid, 500 atoms (FCC 5x5x5, jitter N(0, 0.1)),
    Z = 4, the same local and s+p model and mixing as config 2, 1200 states
    for 2000 electrons, degree 24."""
    rng = np.random.default_rng(seed)
    L = 34.0
    pos = fcc_jittered(L, 5, 0.1, rng)
    na = pos.shape[0]
    return System(
        name="cfg4", n=(120, 120, 120), L=(L, L, L), pos=pos,
        Z=np.full(na, 4.0), rc_loc=np.full(na, 1.0),
        n_states=1200, n_electrons=2000.0, kT=0.01, cheb_degree=24, mix_beta=0.3, kerker_q0=1.0,
        pulay_history=7, pulay_period=2, pulay_restart=1,
        nl_lmax=1, gamma=_gamma(na, 1, seed), rc_nl=1.2, rcut_nl=3.6, seed=seed,
    )


def config5_snapshot(s: int, base_seed: int = 0, n: int = 72, sigma: float = 0.15) -> System:
    """Config-1 cell and physics on an ``n``^3 grid, atoms displaced from the
    config-1 geometry by N(0, sigma) per coordinate drawn with seed ``s``
    (an MD-like snapshot).  Seeds 0..199 train, 200..249 test."""
    base = config1(base_seed, n=n)
    rng = np.random.default_rng([base_seed, 1000 + s])
    pos = np.mod(base.pos + rng.normal(0.0, sigma, base.pos.shape), np.asarray(base.L))
    out = replace(base, pos=pos, name=f"cfg5_s{s}", seed=s)
    return out


def tiny_system(n=(14, 16, 18), L=(4.2, 4.5, 4.8), n_atoms: int = 2, with_nonlocal: bool = True,
                seed: int = 3, n_states: int = 8, Z: float = 2.0) -> System:
    """Small, deliberately non-cubic periodic system for brute-force checks
    (dense diagonalisation of H) and GPU parity on ragged tiles."""
    rng = np.random.default_rng(seed)
    pos = random_positions(L, n_atoms, 1.5, rng)
    na = pos.shape[0]
    return System(
        name="tiny", n=tuple(n), L=tuple(L), pos=pos,
        Z=np.full(na, Z), rc_loc=np.full(na, 0.8),
        n_states=n_states, n_electrons=float(Z * na), kT=0.01, cheb_degree=10,
        nl_lmax=1 if with_nonlocal else -1,
        gamma=_gamma(na, 1, seed) if with_nonlocal else None,
        rc_nl=1.0, rcut_nl=3.0, seed=seed,
    )


def initial_orbitals(nd: int, ns: int, seed: int = 0, dtype=np.float64) -> np.ndarray:
    """Random starting block X0 with entries U(-0.5, 0.5).

    Returned as a C-ordered array of shape (ns, nd): row j is orbital j, which
    is the column-major N_d x N_s layout (leading dimension N_d) used across
    the C ABI."""
    rng = np.random.default_rng([seed, 11])
    return rng.uniform(-0.5, 0.5, (ns, nd)).astype(dtype)


def cnn_initial_weights(seed: int = 0) -> np.ndarray:
    """Starting parameters of the 3 -> 16 -> 16 -> 1 warm-start network
    (flat, float32; layout W1, b1, W2, b2, W3, b3 with W (out, in, 3, 3, 3)):
    He-normal weights N(0, 2 / (27 in)), zero biases, the output layer scaled
    by 0.1."""
    rng = np.random.default_rng([seed, 13])
    parts = []
    for k, (ci, co) in enumerate(((3, 16), (16, 16), (16, 1))):
        W = rng.standard_normal((co, ci, 3, 3, 3)) * np.sqrt(2.0 / (27 * ci))
        if k == 2:
            W *= 0.1
        parts += [W.ravel(), np.zeros(co)]
    return np.concatenate(parts).astype(np.float32)


def initial_orbitals_rows(nd: int, ns: int, seed: int = 0, rows: int = 16):
    """The rows of ``initial_orbitals(nd, ns, seed)`` in consecutive chunks of
    at most ``rows`` (same generator stream, so the values are identical),
    for blocks too large to build on the host at once.  Yields (row0, array)."""
    rng = np.random.default_rng([seed, 11])
    for r0 in range(0, ns, rows):
        k = min(rows, ns - r0)
        yield r0, rng.uniform(-0.5, 0.5, (k, nd))


def config1_spin(seed: int = 0) -> System:
    """Spin-polarised config 1: the config-1 cell and geometry with the last
    atom's charge set to Z = 1 (15 electrons), 12 states per spin, starting
    polarisation zeta0 = 1/15 (one unpaired electron), linear mixing 0.3,
    kT = 0.002 Ha (at config 1's 0.01 Ha the smearing exceeds the exchange
    splitting of the odd electron and the ground state is unpolarised)."""
    s = config1(seed)
    Z = s.Z.copy()
    Z[-1] = 1.0
    return replace(s, name="cfg1s", Z=Z, n_electrons=float(Z.sum()), kT=0.002, spin=2, spin_zeta0=1.0 / 15.0)


def config2_spin(seed: int = 0) -> System:
    """Spin-polarised config 2: the config-2 system with the last atom's
    charge set to Z = 3 (431 electrons), 260 states per spin, starting
    polarisation zeta0 = 1/431, config 2's mixing."""
    s = config2(seed)
    Z = s.Z.copy()
    Z[-1] = 3.0
    return replace(s, name="cfg2s", Z=Z, n_electrons=float(Z.sum()), spin=2, spin_zeta0=1.0 / 431.0)


def initial_orbitals_spin(nd: int, ns: int, seed: int = 0):
    """Starting blocks (up, down) for the spin-polarised form: up is
    ``initial_orbitals(nd, ns, seed)``, down an independent draw."""
    up = initial_orbitals(nd, ns, seed)
    rng = np.random.default_rng([seed, 11, 1])
    return up, rng.uniform(-0.5, 0.5, (ns, nd))


def initial_orbitals_k(nd: int, ns: int, seed: int = 0, q: int = 0) -> np.ndarray:
    """Complex starting block for k-point number q: (ns, nd) with real and
    imaginary parts U(-0.5, 0.5) from their own seeded streams."""
    rng = np.random.default_rng([seed, 11, 2, q])
    re = rng.uniform(-0.5, 0.5, (ns, nd))
    im = rng.uniform(-0.5, 0.5, (ns, nd))
    return re + 1j * im


def monkhorst_pack(L, grid):
    """Monkhorst-Pack k-points of a (n1, n2, n3) grid for an orthorhombic
    cell of lengths L (offsets (2 i - n + 1) / (2 n) of the reciprocal
    vectors: unshifted for odd n, half-shifted for even n), equal weights;
    returns (k (n_k, 3) in 1/Bohr, weights (n_k,))."""
    pts = []
    for a in range(grid[0]):
        for b in range(grid[1]):
            for c in range(grid[2]):
                f = [(2 * i - n + 1) / (2.0 * n) for i, n in zip((a, b, c), grid)]
                pts.append([2.0 * np.pi * f[d] / L[d] for d in range(3)])
    return np.array(pts), np.full(len(pts), 1.0 / len(pts))


CONFIG_NAMES = {
    "cfg1": config1,
    "cfg2": config2,
    "cfg3": config3,
    "cfg4": config4,
    "cfg1s": config1_spin,
    "cfg2s": config2_spin,
}
