"""Shared helpers of the GPU parity tests (inputs from ``workloads``; expected
values from ``oracle``; device work through the C ABI)."""
import sys

import numpy as np
import pytest

import workloads as W


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def ragged_system(nonlocal_part=True, n_states=6):
    """40 x 37 x 13 grid: y-slabs of 16 rows leave a ragged 5-row slab, x is
    not a multiple of 64, z is the smallest allowed length, and the projector
    supports wrap through periodic images."""
    return W.tiny_system(n=(40, 37, 13), L=(12.0, 11.1, 3.9), n_atoms=3, with_nonlocal=nonlocal_part,
                         seed=5, n_states=n_states)


def small_images_system(n_states=6):
    """13 x 14 x 15 grid on a ~4 Bohr cell: every projector overlaps its own
    periodic images."""
    return W.tiny_system(n=(13, 14, 15), L=(4.0, 4.3, 4.6), n_atoms=2, seed=3, n_states=n_states)


def rel_err(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def to_dev(torch, x, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def to_np(t):
    return t.detach().cpu().numpy()
