"""CPU FP64 oracle for the natively periodic FMM — TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code, table or constant generator with the
HIP library under ``paper_2011_07099_amd/``; neither side imports the other.

Contents (each function cites the passage of Gnedin, "Natively Periodic Fast
Multipole Method: Approximating the Optimal Green's Function", that it follows):

* ``green``  — the periodic Green's functions G_X (Eq. 2), G_K (Eq. 1),
  G_S / G_S1 (Sec. 3 ansatz, Eq. 9), the free-space G_0 of the non-periodic
  twin (Eq. 3) and the self-cell value.
* ``conv``   — the exact result the FMM approximates: the periodic convolution
  of the density with G (Eq. 4, "PM with G"), computed three independent ways
  (pairwise brute force, lattice-table direct sum, FFT), PM with G_K, and
  the isolated (non-periodic, zero-padded) convolution with G_0.
* ``fmm``    — a step-by-step FP64 reference of the method (Sec. 2, Eqs. 5-7):
  gridlet anterpolation (P2M/M2M), interaction-zone M2L, interpolation
  (L2L/L2P) and the 27-node near zone; also its non-periodic twin and the
  accelerations taken from the expansion (Sec. 3).
* ``fd``     — periodic 4th-order finite-difference accelerations (Sec. 3).
* ``metric`` — the Green's-function error Delta g of Eq. 3: PM accelerations
  of point sources, the twin's translation, L2 / L_MAX norms.
* ``fit``    — downhill simplex (Sec. 3) for fitting the G_S coefficients.
* ``mlp``    — FP64 network of the learned table correction (Sec. 3-4, G_*).

Parity status: every function is pinned by tests in ``tests/test_oracle_*``
(closed forms, brute force, exact special cases, invariants), except where a
function header says "parity unpinned".
"""
from . import green, conv, fmm, fd, mlp, metric, fit  # noqa: F401
