"""FP64 CPU oracle for the Chebyshev Polynomial Approximation Algorithm (CPAA).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import anything from this package; the GPU
library never calls it and shares no code with it (the only common module is
``graphgen``, which builds inputs and does none of the method's arithmetic).

Everything here is plain, slow and obviously correct: numpy / scipy in float64,
written from the paper (arXiv 2112.01743, "A Parallel PageRank Algorithm For
Undirected Graph"), each function citing the passage it follows.

Parity status: every function is pinned by tests in ``tests/test_oracle.py``
against values the paper prints, closed forms, exact rational arithmetic or
mathematical invariants.  The warm-start network reference is in
``oracle.mpnn``.
"""
from .cpaa_ref import *  # noqa: F401,F403
