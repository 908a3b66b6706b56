"""CPU oracle for the augmented HOC biharmonic solver (FP64, plain and slow).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import, call or run anything under ``oracle/``.  It shares no code with the
HIP implementation; the only module both sides use is the seeded input
generator ``workloads`` (analytic fields, no discretisation arithmetic).

Two tiers:

* ``direct``  -- the plain definition: the coupled HOC linear system of
  Section 2.2 (block system ``eq-coupled``; where the paper is silent or garbled
  the module docstrings state the reading taken) assembled entry by entry in
  FP64 and solved by a sparse LU.
  Also the explicit Schur complement S_h and right-hand side b of Section 2.3.
* ``fast``    -- Algorithm 1 step by step (ConstructSchurRHS, SchurMatVec,
  matrix-free GMRES, recovery of V then U) with library DST-I transforms
  (scipy.fft) as the fast Poisson solver.  Used at sizes the direct tier
  cannot reach, and pinned against the direct tier.

``triharmonic`` is the same pair of tiers for the triharmonic extension of
Sec. 4.2 (Delta^3 u = f, three chained Poisson solves per Schur matvec).

``dst`` holds the naive O(N^2) discrete sine transform, ``stencils`` the
compact operators, ``grid`` node numbering and the layout of Q.
"""
from . import grid, stencils, dst, direct, fast, triharmonic  # noqa: F401
