"""MI355X (gfx950) Chebyshev-filtered subspace iteration for real-space
Kohn-Sham DFT.

The compute path is the HIP library ``libsparc_gpu.so`` (sources in
``csrc/``, C ABI in ``include/sparc_gpu.h``); this package only binds it.
"""
from ._lib import (  # noqa: F401
    EXPORTED,
    SPARC_FP32,
    SPARC_FP64,
    Context,
    SCFReport,
    SCFState,
    SparcError,
    KSCFState,
    SpinSCFState,
    load,
    make_k_state,
    make_spin_state,
    make_state,
)
from .driver import run_scf, run_scf_k, run_scf_spin, scf_forces  # noqa: F401
