"""Plain FP64 CPU oracle for the Chebyshev-filtered subspace iteration (CheFSI)
hot path of real-space Kohn-Sham DFT.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, the smoke check in
``__graft_entry__.py`` and the ``cpu_baseline`` leg of ``bench.py`` use it.
It shares no code, constants or tables with the HIP library; both sides read
the same seeded inputs from ``workloads``, which holds no arithmetic of the
method.

Every function follows the paper's statement of the problem (Kohn-Sham
eigenproblem, Sec. 2 eq. (1); electron density, Sec. 2 eq. (2); the
discretisation, electrostatics and CheFSI described in Sec. 2.1) and, where
the paper is silent, the written-out textbook definition named in its
docstring.  It is written for clarity, not speed: NumPy/SciPy in float64,
with library primitives (FFT, Cholesky, symmetric eigensolver) used as single
steps and no blocking or fusion.

Functions whose results have no pin outside the oracle itself are marked
"parity unpinned" in their docstrings:
  * ``xc.pw92_correlation`` and ``xc.pw92_G`` beyond their high-density
    coefficients and the relation b2 = 2 A b1^2 (the PW92 fit constants a1,
    b1, b3, b4 are not printed in the paper);
  * ``scf.scf`` trajectories away from the fixed point (only GPU <-> oracle
    parity, no outside reference exists for the model systems).
"""
