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
