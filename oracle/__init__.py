"""Plain FP64 CPU oracle for the multi-patch isogeometric multigrid solver.

TEST INFRASTRUCTURE ONLY.  This package is a slow, direct transcription of the
method of Hofer & Takacs, "A parallel multigrid solver for multi-patch
Isogeometric Analysis": the Poisson model problem and its C0 multi-patch
B-spline discretization (Sec. 2), the additive piece-wise smoother and the
multigrid cycle (Sec. 3), Algorithm 1 and the PCG driver (Sec. 4).  It is used
by the tests, by ``__graft_entry__.smoke()`` and by the ``cpu_baseline`` leg of
``bench.py`` to check and time the HIP library; no product code path imports
it, and it shares no code with the library.

Everything is NumPy/SciPy in float64.  Each function cites the passage it
follows.  Readings of passages the paper leaves open are listed in the module
that takes them (look for "Reading").

Parity status per function is stated in the module headers; the only part the
paper does not fix is the interior subspace-corrected mass smoother, whose
construction the paper delegates to its reference [HT:2016] (Sec. 3, first
bullet of the smoother list): its constants are "parity unpinned" against the
paper and are checked only by self-consistency invariants.
"""
