"""Dense symmetric eigensolver of the Rayleigh-Ritz step (Sec. 2.1, CheFSI;
Sec. 4 names this N_s x N_s problem as the cubic part) against
numpy.linalg.eigh, through the C ABI.

Eigenvalues must agree to 1e-12 ||A||; eigenvectors are checked through the
residual ||A V - V diag(lam)|| and the orthogonality ||V^T V - I||, which hold
whatever basis the solver picks inside a degenerate eigenspace.  The
orthogonality bound between eigenvectors of different clusters of an
inverse-iteration solver is eps ||A|| / gap with gap >= 1e-5 ||A|| (the
cluster threshold), about 2e-11; the bound below is 5e-11.
"""
import numpy as np
import pytest

from gpu_helpers import log, require_gpu, to_dev, to_np

pytestmark = pytest.mark.gpu


def _ctx():
    import workloads as W
    from paper_2005_10431_amd import Context
    return Context(W.tiny_system(with_nonlocal=False))


def _random_sym(n, seed):
    a = np.random.default_rng(seed).standard_normal((n, n))
    return 0.5 * (a + a.T)


def _with_spectrum(lam, seed):
    n = len(lam)
    q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((n, n)))
    a = (q * lam) @ q.T
    return 0.5 * (a + a.T)


def _clustered(n, seed):
    rng = np.random.default_rng(seed)
    lam = np.sort(rng.uniform(-1.0, 1.0, n))
    lam[10:14] = lam[10]             # exact 4-fold degeneracy
    lam[40:43] = lam[40] + np.array([0.0, 1e-10, 2e-10])   # near-degenerate triple
    lam[n - 6:] = lam[n - 6] + 1e-6 * np.arange(6)        # tight cluster at the top
    return _with_spectrum(lam, seed + 1)


CASES = {
    "n1": lambda: np.array([[0.37]]),
    "n2": lambda: _random_sym(2, 1),
    "n3": lambda: _random_sym(3, 2),
    "n37": lambda: _random_sym(37, 3),
    "n260_random": lambda: _random_sym(260, 4),
    "n260_clustered": lambda: _clustered(260, 5),
    "diagonal": lambda: np.diag(np.random.default_rng(6).uniform(-2, 2, 50)),
    "block_diagonal": lambda: np.kron(np.eye(5), _random_sym(8, 7)),
    "identity": lambda: np.eye(33),
    "graded": lambda: _with_spectrum(np.geomspace(1e-8, 1.0, 64), 8),
    "n700_random": lambda: _random_sym(700, 9),
    "n4096_random": lambda: _random_sym(4096, 11),   # the largest N the library accepts
}


def _check(case, a, monkeypatch=None, trd_multi_min=None, trd_tail=None):
    torch = require_gpu()
    n = a.shape[0]
    log("subspace_eigh", case, n, "" if trd_multi_min is None
        else f"multi-workgroup reduction from N={trd_multi_min}, one-workgroup tail {trd_tail}")
    if trd_multi_min is not None:
        monkeypatch.setenv("SPARC_GPU_TRD_MULTI_MIN", str(trd_multi_min))
        monkeypatch.setenv("SPARC_GPU_TRD_TAIL", str(trd_tail))
    ctx = _ctx()
    Ad = to_dev(torch, a.T)           # column-major storage
    Vd = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    ed = torch.zeros(n, dtype=torch.float64, device="cuda")
    ctx.subspace_eigh(Ad, Vd, ed)
    lam = to_np(ed)
    V = to_np(Vd).T                   # columns are eigenvectors
    ref = np.linalg.eigvalsh(a)
    anorm = max(np.max(np.abs(ref)), 1e-300)
    eerr = np.max(np.abs(lam - ref)) / anorm
    res = np.max(np.abs(a @ V - V * lam)) / anorm
    orth = np.max(np.abs(V.T @ V - np.eye(n)))
    log(f"  eig {eerr:.2e}  residual {res:.2e}  orth {orth:.2e}")
    assert np.all(np.diff(lam) >= 0.0)
    assert eerr <= 1e-12
    assert res <= 1e-11
    assert orth <= 5e-11


@pytest.mark.parametrize("case", sorted(CASES))
def test_subspace_eigh(case):
    _check(case, CASES[case]())


# The reduction to tridiagonal form spread over many workgroups (used from
# N = 320 on by default), forced down to N = 3 so that one-tile, ragged and
# degenerate cases run through it too, with no one-workgroup tail, a tail of
# 20 rows (the hand-over mid-way) and the default tail of 256 rows; n1200 is
# the cfg4 subspace size.
@pytest.mark.parametrize("tail", [0, 20, 256])
@pytest.mark.parametrize("case", ["n3", "n37", "n260_clustered", "graded", "block_diagonal", "identity",
                                  "n700_random", "n1200_clustered"])
def test_subspace_eigh_multi_workgroup_reduction(case, tail, monkeypatch):
    a = _clustered(1200, 10) if case == "n1200_clustered" else CASES[case]()
    _check(case, a, monkeypatch, trd_multi_min=3, trd_tail=tail)

