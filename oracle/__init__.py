"""FP64 CPU oracle for geometric adaptive smoothed-aggregation multigrid on DG
matrices (Pan, Lindsey & Persson, arXiv 2504.13373).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
restatement of the method, written from the paper, used to check the HIP
library.  Only the tests, the smoke check and the benchmark's CPU-baseline leg
may import it; the product path never does.  It shares no code with the HIP
library; both take their inputs from the seeded generators in ``workloads``.

Modules
-------
rng      counter-based SplitMix64 stream (power-iteration start vectors)
rcb      recursive coordinate bisection hierarchy (stand-in for the METIS
         splits of Section 4.1)
amg      setup (Algorithm 5: Algorithm 4 + eq:omega, eq:bsmooth, eq:splitB_dg,
         eq:sik, eq:TR0, Galerkin product) and the V-cycle (Algorithms 1, 2)
krylov   PCG, right-preconditioned FGMRES(m) with CGS2, iterative refinement

Every function states the passage it follows.  Readings of passages that are
silent or garbled are listed in the docstrings of the functions concerned.
"""
