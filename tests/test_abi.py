"""Host-side checks of the C ABI: the library builds, loads and exports every
entry point that ``include/sparc_gpu.h`` declares (no compute calls: these run
without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sparc_gpu.h")
LIB = os.path.join(ROOT, "paper_2005_10431_amd", "libsparc_gpu.so")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sparc_gpu_[a-zA-Z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2005_10431_amd.build import build
        build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_hot_path_calls():
    fns = declared_functions()
    for name in ["sparc_gpu_apply_H", "sparc_gpu_chebyshev_filter", "sparc_gpu_rayleigh_ritz",
                 "sparc_gpu_density", "sparc_gpu_scf_step"]:
        assert name in fns


def test_library_exports_every_declared_symbol(lib):
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing


def test_binding_lists_every_declared_symbol():
    from paper_2005_10431_amd._lib import EXPORTED
    assert sorted(EXPORTED) == declared_functions()


def test_binding_struct_layout_matches_header():
    """Field order and sizes of the ctypes mirrors match the C structs."""
    from paper_2005_10431_amd import _lib
    txt = open(HEADER).read()
    for cname, py in (("sparc_gpu_system", _lib.System), ("sparc_gpu_scf_state", _lib.SCFState),
                      ("sparc_gpu_scf_spin_state", _lib.SpinSCFState), ("sparc_gpu_scf_k_state", _lib.KSCFState),
                      ("sparc_gpu_scf_report", _lib.SCFReport)):
        body = re.search(r"typedef struct \{([^{}]*)\}\s*" + cname + ";", txt).group(1)
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        names = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            parts = decl.replace("*", " ").split()
            # "double band, exc, vxc_dc" declares several names
            tail = decl.split(None, 1)[1] if " " in decl else decl
            for nm in tail.split(","):
                nm = nm.replace("*", "").strip()
                nm = re.sub(r"\[.*\]", "", nm).split()[-1]
                names.append(nm)
        assert [f[0] for f in py._fields_] == names, cname


def test_null_context_is_rejected_without_a_device(lib):
    lib.sparc_gpu_destroy.restype = ctypes.c_int
    lib.sparc_gpu_destroy.argtypes = [ctypes.c_void_p]
    assert lib.sparc_gpu_destroy(None) == 1          # SPARC_ERR_ARG
    lib.sparc_gpu_create.restype = ctypes.c_int
    lib.sparc_gpu_create.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    assert lib.sparc_gpu_create(None, None, None) == 1


def _system_struct(n, half_order):
    """A valid one-atom local-only system on an n[0] x n[1] x n[2] grid."""
    from paper_2005_10431_amd import _lib
    s = _lib.System()
    for d in range(3):
        s.n[d] = n[d]
        s.L[d] = 0.3 * n[d]
    s.fd_half_order = half_order
    keep = [(ctypes.c_double * 3)(0.5, 0.5, 0.5), (ctypes.c_double * 1)(2.0), (ctypes.c_double * 1)(0.8)]
    s.n_atoms = 1
    s.pos = ctypes.cast(keep[0], ctypes.POINTER(ctypes.c_double))
    s.Z = ctypes.cast(keep[1], ctypes.POINTER(ctypes.c_double))
    s.rc_loc = ctypes.cast(keep[2], ctypes.POINTER(ctypes.c_double))
    s.nl_lmax = -1
    s.n_states = 4
    s.n_electrons = 2.0
    s.kT = 0.01
    s.rho_floor = 1e-14
    s.sad_width = 1.0
    return s, keep


@pytest.mark.parametrize("n, half_order", [((5, 5, 5), 2), ((12, 20, 20), 6), ((20, 12, 20), 3),
                                           ((20, 20, 12), 1), ((13, 13, 13), 7), ((13, 13, 13), 0)])
def test_create_rejects_grids_below_the_kernel_half_width(lib, n, half_order):
    """Every axis needs 13 points (twice the kernels' stencil half-width of 6,
    plus one) whatever the order; lower orders do not relax it.  Validation
    runs before any device call, so this needs no GPU."""
    s, keep = _system_struct(n, half_order)
    lib.sparc_gpu_create.restype = ctypes.c_int
    lib.sparc_gpu_create.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    out = ctypes.c_void_p(7)
    assert lib.sparc_gpu_create(ctypes.byref(s), None, ctypes.byref(out)) == 1   # SPARC_ERR_ARG
    assert out.value is None
