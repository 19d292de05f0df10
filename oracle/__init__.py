"""CPU FP64 oracle for group-patch joint compression and the compressed Wave
operator (arXiv 2601.05418).

TEST INFRASTRUCTURE, NOT PART OF THE LIBRARY.  A plain, slow, NumPy complex128
reference written from the paper: Section 2.2 (Eqs. 1-4, the signal model),
Section 2.3 (hybrid-space factorisation, periodic grouping), Section 2.4
(Eqs. 6-15, compression), Sections 3.1 and 5 (general, nonlinear modulation
maps and compressed readout matrices stored per phase-encode column), 3D
volumes with two phase-encode dimensions (Table S2, Figs. 8-9),
Section 3.4 (Eqs. 16-17, reconstruction algorithms #1 and #2 and the NRMSE
metric).  It may be imported only by ``tests/``, by the smoke check and
by the benchmark's CPU-baseline leg.  It shares no code with the HIP path and
imports nothing from it; inputs reach it as arrays.

Parity status of each part is recorded in the module docstrings:
every function is pinned by a CPU test against something other than itself,
except the exact FISTA iterate after many iterations and the reduced-precision
error values ("parity unpinned": they are checked only against this oracle's
same-schedule run and the stated error bounds).
"""
from . import compression, encoding, explicit, hybrid, solvers, volume  # noqa: F401
