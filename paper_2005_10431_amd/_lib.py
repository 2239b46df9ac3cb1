"""ctypes binding of ``libsparc_gpu.so`` (declared in ``include/sparc_gpu.h``).

Argument marshalling only: every computation runs in the library's HIP
kernels.  Device buffers are torch tensors on the current HIP device; their
raw addresses cross the C ABI.  Loading fails loudly when the shared library
has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsparc_gpu.so")

SPARC_FP64 = 0
SPARC_FP32 = 1

STATUS = {
    0: "SPARC_OK",
    1: "SPARC_ERR_ARG",
    2: "SPARC_ERR_HIP",
    3: "SPARC_ERR_NOMEM",
    4: "SPARC_ERR_NOT_SPD",
    5: "SPARC_ERR_EIG",
    6: "SPARC_ERR_FERMI",
    7: "SPARC_ERR_NOCONV",
    8: "SPARC_ERR_NONFINITE",
    9: "SPARC_ERR_SINGULAR",
}

PULAY_MAX = 10

EXPORTED = [
    "sparc_gpu_create",
    "sparc_gpu_destroy",
    "sparc_gpu_last_error",
    "sparc_gpu_grid_size",
    "sparc_gpu_dV",
    "sparc_gpu_set_veff",
    "sparc_gpu_apply_H",
    "sparc_gpu_chebyshev_filter",
    "sparc_gpu_chebyshev_filter_noalloc",
    "sparc_gpu_rayleigh_ritz",
    "sparc_gpu_subspace_eigh",
    "sparc_gpu_density",
    "sparc_gpu_occupations",
    "sparc_gpu_potential",
    "sparc_gpu_pseudocharge",
    "sparc_gpu_sad_density",
    "sparc_gpu_sad_density_spin",
    "sparc_gpu_spectrum_bounds",
    "sparc_gpu_mix",
    "sparc_gpu_potential_spin",
    "sparc_gpu_occupations_spin",
    "sparc_gpu_scf_step_spin",
    "sparc_gpu_forces",
    "sparc_gpu_apply_H_k",
    "sparc_gpu_chebyshev_filter_k",
    "sparc_gpu_rayleigh_ritz_k",
    "sparc_gpu_spectrum_bounds_k",
    "sparc_gpu_scf_step_k",
    "sparc_gpu_scf_step",
    "sparc_gpu_final_rr_fp64",
    "sparc_gpu_profile",
    "sparc_gpu_profile_read",
    "sparc_gpu_features",
    "sparc_gpu_cnn_forward",
    "sparc_gpu_cnn_backward",
    "sparc_gpu_adam_step",
    "sparc_gpu_warm_start",
]

CNN_NPARAMS = 8673


class SparcError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class System(C.Structure):
    _fields_ = [
        ("n", C.c_int * 3),
        ("L", C.c_double * 3),
        ("fd_half_order", C.c_int),
        ("n_atoms", C.c_int),
        ("pos", C.POINTER(C.c_double)),
        ("Z", C.POINTER(C.c_double)),
        ("rc_loc", C.POINTER(C.c_double)),
        ("nl_lmax", C.c_int),
        ("gamma", C.POINTER(C.c_double)),
        ("rc_nl", C.c_double),
        ("rcut_nl", C.c_double),
        ("n_states", C.c_int),
        ("n_electrons", C.c_double),
        ("kT", C.c_double),
        ("rho_floor", C.c_double),
        ("sad_width", C.c_double),
    ]


class SCFState(C.Structure):
    _fields_ = [
        ("d_rho_in", C.c_void_p),
        ("d_X", C.c_void_p),
        ("ldx", C.c_long),
        ("prec", C.c_int),
        ("cheb_degree", C.c_int),
        ("n_first", C.c_int),
        ("mix_beta", C.c_double),
        ("kerker_q0", C.c_double),
        ("pulay_history", C.c_int),
        ("pulay_period", C.c_int),
        ("pulay_restart", C.c_int),
        ("d_pulay", C.c_void_p),
        ("iter", C.c_int),
        ("d_eig", C.c_void_p),
        ("d_occ", C.c_void_p),
        ("d_rho_out", C.c_void_p),
        ("bounds", C.c_double * 3),
    ]


class SpinSCFState(C.Structure):
    _fields_ = [
        ("d_rho_in", C.c_void_p),
        ("d_X_up", C.c_void_p),
        ("d_X_dn", C.c_void_p),
        ("ldx", C.c_long),
        ("prec", C.c_int),
        ("cheb_degree", C.c_int),
        ("n_first", C.c_int),
        ("mix_beta", C.c_double),
        ("kerker_q0", C.c_double),
        ("pulay_history", C.c_int),
        ("pulay_period", C.c_int),
        ("pulay_restart", C.c_int),
        ("d_pulay", C.c_void_p),
        ("iter", C.c_int),
        ("d_eig", C.c_void_p),
        ("d_occ", C.c_void_p),
        ("d_rho_out", C.c_void_p),
        ("bounds", C.c_double * 6),
    ]


class KSCFState(C.Structure):
    _fields_ = [
        ("n_k", C.c_int),
        ("kpts", C.POINTER(C.c_double)),
        ("kweights", C.POINTER(C.c_double)),
        ("d_X", C.POINTER(C.c_void_p)),
        ("ldx", C.c_long),
        ("prec", C.c_int),
        ("cheb_degree", C.c_int),
        ("n_first", C.c_int),
        ("mix_beta", C.c_double),
        ("kerker_q0", C.c_double),
        ("pulay_history", C.c_int),
        ("pulay_period", C.c_int),
        ("pulay_restart", C.c_int),
        ("d_pulay", C.c_void_p),
        ("d_rho_in", C.c_void_p),
        ("iter", C.c_int),
        ("d_eig", C.c_void_p),
        ("d_occ", C.c_void_p),
        ("d_rho_out", C.c_void_p),
        ("bounds", C.POINTER(C.c_double)),
    ]


class SCFReport(C.Structure):
    _fields_ = [
        ("free_energy", C.c_double),
        ("band", C.c_double),
        ("exc", C.c_double),
        ("vxc_dc", C.c_double),
        ("elec", C.c_double),
        ("self_energy", C.c_double),
        ("overlap", C.c_double),
        ("entropy", C.c_double),
        ("mu", C.c_double),
        ("residual", C.c_double),
        ("t_potential_ms", C.c_double),
        ("t_filter_ms", C.c_double),
        ("t_rr_ms", C.c_double),
        ("t_density_ms", C.c_double),
        ("t_total_ms", C.c_double),
        ("n_passes", C.c_int),
        ("iter", C.c_int),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load(path: str = LIB_PATH):
    """Load the shared library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} not found: build it with `python -m paper_2005_10431_amd.build` "
            "(there is no fallback implementation)")
    lib = C.CDLL(path)
    vp, i, l, d = C.c_void_p, C.c_int, C.c_long, C.c_double
    sig = {
        "sparc_gpu_create": ([C.POINTER(System), vp, C.POINTER(vp)], i),
        "sparc_gpu_destroy": ([vp], i),
        "sparc_gpu_last_error": ([vp], C.c_char_p),
        "sparc_gpu_grid_size": ([vp], l),
        "sparc_gpu_dV": ([vp], d),
        "sparc_gpu_set_veff": ([vp, vp], i),
        "sparc_gpu_apply_H": ([vp, i, vp, vp, i, l], i),
        "sparc_gpu_chebyshev_filter": ([vp, i, vp, vp, i, l, i, d, d, d], i),
        "sparc_gpu_chebyshev_filter_noalloc": ([vp, i, vp, vp, i, l, i, d, d, d], i),
        "sparc_gpu_rayleigh_ritz": ([vp, i, vp, i, l, vp], i),
        "sparc_gpu_subspace_eigh": ([vp, vp, i, vp, vp], i),
        "sparc_gpu_density": ([vp, i, vp, i, l, vp, vp], i),
        "sparc_gpu_occupations": ([vp, vp, i, vp, vp], i),
        "sparc_gpu_potential": ([vp, vp, vp, vp, vp, vp], i),
        "sparc_gpu_pseudocharge": ([vp, vp, C.POINTER(d), C.POINTER(d)], i),
        "sparc_gpu_sad_density": ([vp, vp], i),
        "sparc_gpu_sad_density_spin": ([vp, C.c_double, vp], i),
        "sparc_gpu_spectrum_bounds": ([vp, C.POINTER(d), C.POINTER(d)], i),
        "sparc_gpu_mix": ([vp, vp, vp, i, d, d, i, i, i, vp, i], i),
        "sparc_gpu_potential_spin": ([vp, vp, vp, vp, vp, vp], i),
        "sparc_gpu_occupations_spin": ([vp, vp, i, vp, vp], i),
        "sparc_gpu_scf_step_spin": ([vp, C.POINTER(SpinSCFState), C.POINTER(SCFReport)], i),
        "sparc_gpu_forces": ([vp, vp, i, C.POINTER(vp), i, i, l, vp, vp], i),
        "sparc_gpu_apply_H_k": ([vp, C.POINTER(d), i, vp, vp, i, l], i),
        "sparc_gpu_chebyshev_filter_k": ([vp, C.POINTER(d), i, vp, vp, i, l, i, d, d, d], i),
        "sparc_gpu_rayleigh_ritz_k": ([vp, C.POINTER(d), i, vp, i, l, vp], i),
        "sparc_gpu_spectrum_bounds_k": ([vp, C.POINTER(d), C.POINTER(d), C.POINTER(d)], i),
        "sparc_gpu_scf_step_k": ([vp, C.POINTER(KSCFState), C.POINTER(SCFReport)], i),
        "sparc_gpu_scf_step": ([vp, C.POINTER(SCFState), C.POINTER(SCFReport)], i),
        "sparc_gpu_final_rr_fp64": ([vp, C.POINTER(SCFState), vp, l, C.POINTER(SCFReport)], i),
        "sparc_gpu_profile": ([vp, i], i),
        "sparc_gpu_profile_read": ([vp, i, C.POINTER(d), C.POINTER(l)], i),
        "sparc_gpu_features": ([vp, C.POINTER(d), vp], i),
        "sparc_gpu_cnn_forward": ([vp, vp, vp, vp, vp], i),
        "sparc_gpu_cnn_backward": ([vp, vp, vp, vp, vp, vp, vp, vp], i),
        "sparc_gpu_adam_step": ([vp, vp, vp, vp, vp, i, i, d, d, d, d], i),
        "sparc_gpu_warm_start": ([vp, vp, d, vp, C.POINTER(i)], i),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _ptr(t):
    """Device address of a torch tensor (or None -> NULL)."""
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def _prec_of(t):
    import torch
    if t.dtype == torch.float64:
        return SPARC_FP64
    if t.dtype == torch.float32:
        return SPARC_FP32
    raise TypeError(f"unsupported block dtype {t.dtype}")


def _block(X):
    """(ncol, ld) of a block stored as a torch tensor of shape (ncol, ld)."""
    if X.dim() != 2 or X.stride(1) != 1:
        raise ValueError("blocks are (ncol, ld) tensors with unit stride along the grid")
    return X.shape[0], X.stride(0)


class Context:
    """One library context (``sparc_gpu_ctx``) for a ``workloads.System``."""

    def __init__(self, system, stream=None):
        import numpy as np
        import torch
        self.lib = load()
        s = system
        self._pos = np.ascontiguousarray(s.pos, dtype=np.float64).ravel()
        self._Z = np.ascontiguousarray(s.Z, dtype=np.float64)
        self._rc = np.ascontiguousarray(s.rc_loc, dtype=np.float64)
        self._gamma = (np.ascontiguousarray(s.gamma, dtype=np.float64).ravel()
                       if s.nl_lmax >= 0 and s.gamma is not None else None)
        dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None
        cs = System()
        cs.n = (C.c_int * 3)(*[int(v) for v in s.n])
        cs.L = (C.c_double * 3)(*[float(v) for v in s.L])
        cs.fd_half_order = int(s.fd_half_order)
        cs.n_atoms = int(s.n_atoms)
        cs.pos = dp(self._pos)
        cs.Z = dp(self._Z)
        cs.rc_loc = dp(self._rc)
        cs.nl_lmax = int(s.nl_lmax)
        cs.gamma = dp(self._gamma)
        cs.rc_nl = float(s.rc_nl)
        cs.rcut_nl = float(s.rcut_nl)
        cs.n_states = int(s.n_states)
        cs.n_electrons = float(s.n_electrons)
        cs.kT = float(s.kT)
        cs.rho_floor = float(s.rho_floor)
        cs.sad_width = float(s.sad_width)
        self.system = s
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = C.c_void_p()
        st = self.lib.sparc_gpu_create(C.byref(cs), C.c_void_p(stream.cuda_stream), C.byref(h))
        if st != 0:
            raise SparcError(st, "sparc_gpu_create failed")
        self.h = h
        self.nd = int(self.lib.sparc_gpu_grid_size(h))
        self.dV = float(self.lib.sparc_gpu_dV(h))

    def close(self):
        if getattr(self, "h", None):
            self.lib.sparc_gpu_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != 0:
            msg = self.lib.sparc_gpu_last_error(self.h)
            raise SparcError(st, msg.decode() if msg else "")

    # ---- calls (same names as the C ABI) ----
    def set_veff(self, veff):
        self._check(self.lib.sparc_gpu_set_veff(self.h, _ptr(veff)))

    def apply_H(self, X, Y):
        ncol, ld = _block(X)
        self._check(self.lib.sparc_gpu_apply_H(self.h, _prec_of(X), _ptr(X), _ptr(Y), ncol, ld))

    def chebyshev_filter(self, X, work, degree, a, b, a0):
        ncol, ld = _block(X)
        self._check(self.lib.sparc_gpu_chebyshev_filter(self.h, _prec_of(X), _ptr(X), _ptr(work), ncol, ld,
                                                        int(degree), float(a), float(b), float(a0)))

    def chebyshev_filter_noalloc(self, X, work, degree, a, b, a0):
        """The filter with its scratch in the library's fixed device array."""
        ncol, ld = _block(X)
        self._check(self.lib.sparc_gpu_chebyshev_filter_noalloc(self.h, _prec_of(X), _ptr(X), _ptr(work), ncol,
                                                                ld, int(degree), float(a), float(b), float(a0)))

    def rayleigh_ritz(self, X, eig):
        ncol, ld = _block(X)
        self._check(self.lib.sparc_gpu_rayleigh_ritz(self.h, _prec_of(X), _ptr(X), ncol, ld, _ptr(eig)))

    def subspace_eigh(self, A, V, eig):
        """A: (n, n) float64 device tensor (destroyed; symmetric)."""
        n = A.shape[0]
        self._check(self.lib.sparc_gpu_subspace_eigh(self.h, _ptr(A), int(n), _ptr(V), _ptr(eig)))

    def density(self, X, occ, rho):
        ncol, ld = _block(X)
        self._check(self.lib.sparc_gpu_density(self.h, _prec_of(X), _ptr(X), ncol, ld, _ptr(occ), _ptr(rho)))

    def occupations(self, eig, occ, mu=None):
        self._check(self.lib.sparc_gpu_occupations(self.h, _ptr(eig), int(eig.numel()), _ptr(occ), _ptr(mu)))

    def potential(self, rho, phi=None, exc=None, vxc=None, veff=None):
        self._check(self.lib.sparc_gpu_potential(self.h, _ptr(rho), _ptr(phi), _ptr(exc), _ptr(vxc), _ptr(veff)))

    def pseudocharge(self, b=None):
        es, ec = C.c_double(), C.c_double()
        self._check(self.lib.sparc_gpu_pseudocharge(self.h, _ptr(b), C.byref(es), C.byref(ec)))
        return es.value, ec.value

    def sad_density(self, rho):
        self._check(self.lib.sparc_gpu_sad_density(self.h, _ptr(rho)))

    def sad_density_spin(self, zeta0, rho2):
        """rho2: (2 N_d,) float64, up then down."""
        self._check(self.lib.sparc_gpu_sad_density_spin(self.h, float(zeta0), _ptr(rho2)))

    def spectrum_bounds(self):
        lo, hi = C.c_double(), C.c_double()
        self._check(self.lib.sparc_gpu_spectrum_bounds(self.h, C.byref(lo), C.byref(hi)))
        return lo.value, hi.value

    def mix(self, rho_in, rho_out, beta, kerker_q0=0.0, pulay_history=0, pulay_period=1, restart=False,
            hist=None, iter=0, n_spin=1):
        """rho_in (updated in place), rho_out: (n_spin N_d,) float64; hist:
        ((2 m + 2) n_spin N_d,) float64 history buffer when pulay_history = m > 0."""
        self._check(self.lib.sparc_gpu_mix(self.h, _ptr(rho_in), _ptr(rho_out), int(n_spin), float(beta),
                                           float(kerker_q0), int(pulay_history), int(pulay_period),
                                           1 if restart else 0, _ptr(hist), int(iter)))

    def potential_spin(self, rho, phi=None, exc=None, vxc=None, veff=None):
        """rho: (2 N_d,) up then down; vxc, veff: (2 N_d,)."""
        self._check(self.lib.sparc_gpu_potential_spin(self.h, _ptr(rho), _ptr(phi), _ptr(exc), _ptr(vxc),
                                                       _ptr(veff)))

    def occupations_spin(self, eig, occ, mu=None):
        """eig, occ: (2 ncol,) float64, up then down."""
        self._check(self.lib.sparc_gpu_occupations_spin(self.h, _ptr(eig), int(eig.numel()) // 2, _ptr(occ),
                                                        _ptr(mu)))

    def forces(self, phi, blocks, occ, out):
        """phi: (N_d,) float64; blocks: list of 0-2 orbital blocks (ncol, ld)
        of one dtype; occ: (len(blocks) ncol,) float64 weights; out: (n_atoms, 3)
        float64, overwritten."""
        n = len(blocks)
        ptrs = (C.c_void_p * max(n, 1))(*[b.data_ptr() for b in blocks])
        ncol, ld, prec = (0, 0, SPARC_FP64)
        if n:
            ncol, ld = _block(blocks[0])
            prec = _prec_of(blocks[0])
            for b in blocks[1:]:
                if _block(b) != (ncol, ld) or _prec_of(b) != prec:
                    raise ValueError("orbital blocks must share shape, leading dimension and dtype")
        self._check(self.lib.sparc_gpu_forces(self.h, _ptr(phi), prec, ptrs, n, ncol, ld, _ptr(occ), _ptr(out)))

    # ---- Bloch k-points: blocks of columns [Re z; Im z], shape (ncol, >= 2 N_d)
    @staticmethod
    def _k(k):
        return (C.c_double * 3)(*[float(v) for v in k])

    def apply_H_k(self, k, X, Y):
        ncol, ld = _block(X)
        self._check(self.lib.sparc_gpu_apply_H_k(self.h, self._k(k), _prec_of(X), _ptr(X), _ptr(Y), ncol, ld))

    def chebyshev_filter_k(self, k, X, work, degree, a, b, a0):
        ncol, ld = _block(X)
        self._check(self.lib.sparc_gpu_chebyshev_filter_k(self.h, self._k(k), _prec_of(X), _ptr(X), _ptr(work), ncol,
                                                          ld, int(degree), float(a), float(b), float(a0)))

    def rayleigh_ritz_k(self, k, X, eig):
        ncol, ld = _block(X)
        self._check(self.lib.sparc_gpu_rayleigh_ritz_k(self.h, self._k(k), _prec_of(X), _ptr(X), ncol, ld,
                                                       _ptr(eig)))

    def spectrum_bounds_k(self, k):
        lo, hi = C.c_double(), C.c_double()
        self._check(self.lib.sparc_gpu_spectrum_bounds_k(self.h, self._k(k), C.byref(lo), C.byref(hi)))
        return lo.value, hi.value

    def scf_step_k(self, state) -> dict:
        rep = SCFReport()
        self._check(self.lib.sparc_gpu_scf_step_k(self.h, C.byref(state), C.byref(rep)))
        return rep.as_dict()

    def scf_step_spin(self, state) -> dict:
        rep = SCFReport()
        self._check(self.lib.sparc_gpu_scf_step_spin(self.h, C.byref(state), C.byref(rep)))
        return rep.as_dict()

    def scf_step(self, state: SCFState) -> dict:
        rep = SCFReport()
        self._check(self.lib.sparc_gpu_scf_step(self.h, C.byref(state), C.byref(rep)))
        return rep.as_dict()

    def profile(self, enable: bool):
        self._check(self.lib.sparc_gpu_profile(self.h, 1 if enable else 0))

    def profile_read(self, kernel_id: int):
        ms, n = C.c_double(), C.c_long()
        self._check(self.lib.sparc_gpu_profile_read(self.h, int(kernel_id), C.byref(ms), C.byref(n)))
        return ms.value, n.value

    # ---- learned initial density
    def features(self, feat, widths=(0.5, 1.0, 2.0)):
        """feat: (3, N_d) float32 device tensor."""
        w = (C.c_double * 3)(*[float(x) for x in widths])
        self._check(self.lib.sparc_gpu_features(self.h, w, _ptr(feat)))

    def cnn_forward(self, w, feat, act, rho):
        """w: (8673,) float32; feat: (3, N_d) float32; act: (33, N_d) float32
        scratch; rho: (N_d,) float64 out."""
        self._check(self.lib.sparc_gpu_cnn_forward(self.h, _ptr(w), _ptr(feat), _ptr(act), _ptr(rho)))

    def cnn_backward(self, w, feat, act, rho, target, grad, loss=None):
        self._check(self.lib.sparc_gpu_cnn_backward(self.h, _ptr(w), _ptr(feat), _ptr(act), _ptr(rho),
                                                    _ptr(target), _ptr(grad), _ptr(loss)))

    def adam_step(self, w, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self._check(self.lib.sparc_gpu_adam_step(self.h, _ptr(w), _ptr(grad), _ptr(m), _ptr(v), int(w.numel()),
                                                 int(t), float(lr), float(beta1), float(beta2), float(eps)))

    def warm_start(self, w, rho, max_l1=0.5) -> bool:
        used = C.c_int(0)
        self._check(self.lib.sparc_gpu_warm_start(self.h, _ptr(w), float(max_l1), _ptr(rho), C.byref(used)))
        return bool(used.value)

    def final_rr_fp64(self, state: SCFState, X64) -> dict:
        rep = SCFReport()
        ncol, ld = _block(X64)
        self._check(self.lib.sparc_gpu_final_rr_fp64(self.h, C.byref(state), _ptr(X64), ld, C.byref(rep)))
        return rep.as_dict()


def make_state(rho_in, X, eig, occ, degree, n_first=4, beta=0.3, rho_out=None, kerker_q0=0.0,
               pulay_history=0, pulay_period=1, pulay_restart=False, pulay_hist=None) -> SCFState:
    """pulay_hist: ((2 m + 2) N_d,) float64 device tensor when
    pulay_history = m > 0 (the caller keeps it alive with the state)."""
    st = SCFState()
    st.d_rho_in = rho_in.data_ptr()
    st.d_X = X.data_ptr()
    st.ldx = X.stride(0)
    st.prec = _prec_of(X)
    st.cheb_degree = int(degree)
    st.n_first = int(n_first)
    st.mix_beta = float(beta)
    st.kerker_q0 = float(kerker_q0)
    st.pulay_history = int(pulay_history)
    st.pulay_period = int(pulay_period)
    st.pulay_restart = 1 if pulay_restart else 0
    st.d_pulay = pulay_hist.data_ptr() if pulay_hist is not None else None
    st.iter = 0
    st.d_eig = eig.data_ptr()
    st.d_occ = occ.data_ptr()
    st.d_rho_out = rho_out.data_ptr() if rho_out is not None else None
    st.bounds = (C.c_double * 3)(0.0, 0.0, 0.0)
    return st


def make_spin_state(rho_in, X_up, X_dn, eig, occ, degree, n_first=4, beta=0.3, rho_out=None, kerker_q0=0.0,
                    pulay_history=0, pulay_period=1, pulay_restart=False, pulay_hist=None) -> SpinSCFState:
    """rho_in: (2 N_d,) float64 (up, down); X_up, X_dn: (n_states, ld) blocks of
    one dtype and ld; eig, occ: (2 n_states,) float64; pulay_hist:
    ((2 m + 2) 2 N_d,) float64 when pulay_history = m > 0."""
    if X_up.stride(0) != X_dn.stride(0) or X_up.dtype != X_dn.dtype:
        raise ValueError("spin blocks must share dtype and leading dimension")
    st = SpinSCFState()
    st.d_rho_in = rho_in.data_ptr()
    st.d_X_up = X_up.data_ptr()
    st.d_X_dn = X_dn.data_ptr()
    st.ldx = X_up.stride(0)
    st.prec = _prec_of(X_up)
    st.cheb_degree = int(degree)
    st.n_first = int(n_first)
    st.mix_beta = float(beta)
    st.kerker_q0 = float(kerker_q0)
    st.pulay_history = int(pulay_history)
    st.pulay_period = int(pulay_period)
    st.pulay_restart = 1 if pulay_restart else 0
    st.d_pulay = pulay_hist.data_ptr() if pulay_hist is not None else None
    st.iter = 0
    st.d_eig = eig.data_ptr()
    st.d_occ = occ.data_ptr()
    st.d_rho_out = rho_out.data_ptr() if rho_out is not None else None
    st.bounds = (C.c_double * 6)(*([0.0] * 6))
    return st


def make_k_state(rho_in, blocks, kpts, kweights, eig, occ, degree, n_first=4, beta=0.3, rho_out=None,
                 kerker_q0=0.0, pulay_history=0, pulay_period=1, pulay_restart=False, pulay_hist=None) -> KSCFState:
    """blocks: list of n_k device tensors (2 n_states, ld >= 2 N_d) of one
    dtype and ld; kpts (n_k, 3), kweights (n_k,) host arrays; eig, occ:
    (n_k 2 n_states,) float64.  The host arrays the state points to are kept
    on the returned object."""
    import numpy as np
    n = len(blocks)
    ld = blocks[0].stride(0)
    for b in blocks:
        if b.stride(0) != ld or b.dtype != blocks[0].dtype:
            raise ValueError("k-point blocks must share dtype and leading dimension")
    st = KSCFState()
    st._kp = (C.c_double * (3 * n))(*[float(v) for v in np.asarray(kpts, dtype=np.float64).ravel()])
    st._kw = (C.c_double * n)(*[float(v) for v in kweights])
    st._px = (C.c_void_p * n)(*[b.data_ptr() for b in blocks])
    st._bd = (C.c_double * (3 * n))(*([0.0] * (3 * n)))
    st.n_k = n
    st.kpts = C.cast(st._kp, C.POINTER(C.c_double))
    st.kweights = C.cast(st._kw, C.POINTER(C.c_double))
    st.d_X = C.cast(st._px, C.POINTER(C.c_void_p))
    st.ldx = ld
    st.prec = _prec_of(blocks[0])
    st.cheb_degree = int(degree)
    st.n_first = int(n_first)
    st.mix_beta = float(beta)
    st.kerker_q0 = float(kerker_q0)
    st.pulay_history = int(pulay_history)
    st.pulay_period = int(pulay_period)
    st.pulay_restart = 1 if pulay_restart else 0
    st.d_pulay = pulay_hist.data_ptr() if pulay_hist is not None else None
    st.d_rho_in = rho_in.data_ptr()
    st.iter = 0
    st.d_eig = eig.data_ptr()
    st.d_occ = occ.data_ptr()
    st.d_rho_out = rho_out.data_ptr() if rho_out is not None else None
    st.bounds = C.cast(st._bd, C.POINTER(C.c_double))
    return st
