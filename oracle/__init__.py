"""Plain FP64 CPU oracle for the HDG trace multigrid solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call,
link or execute anything in this package: only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py``
use it.  It shares no code with the HIP library; it takes every input as
plain arrays so that the seeded generators are the only common piece.

Layout of the package (each function cites the passage of the paper it
follows):

* ``refelem``  -- 1D Gauss-Lobatto-Legendre nodes, Gauss rules, Lagrange
  bases (the nodal spaces of Sec. 2).
* ``hdg``      -- structured mesh numbering, the HDG local problem
  (eqs. HDG, HDG_flux), static condensation into the trace system
  A lambda = g (eq. trace_linear_system), local recovery, the monolithic
  (uncondensed) system and error norms.
* ``mg``       -- the multigrid hierarchy of Sec. 3: p-coarsening
  (Sec. 3.1.1), h-coarsening by agglomeration (eq. trace_partition),
  prolongation (eqs. n_1_Ik, n_g1_Ik), restriction (eqs. n_1_Qk, n_g1_Qk),
  Galerkin coarse operators (eqs. coarse, Akm1, ANm1), block-Jacobi
  smoothing (Sec. 3.3 and Sec. 4.1), local correction (eq.
  localCorrection), the V-cycle (Algorithm 1) and the outer iterations
  (fixed point, CG, GMRES; Sec. 3.6 and Sec. 4).
* ``ipdg``     -- the hybridized interior penalty family (SIPG-H, IIPG-H,
  NIPG-H; eqs. IPDG_flux, SIPG_H, IPG_H): element matrices, static
  condensation into the same trace system, recovery of u and
  q = -kappa grad u, and the uncondensed system.
* ``rth``      -- the hybridized Raviart-Thomas mixed method (RT_k-H on
  squares, eqs. mixed_local1, mixed_local2) and multinumerics (RT-H and an
  IPDG scheme element by element in one trace system, Sec. 4.6).
* ``unstructured`` -- HDG on P^k triangles of an unstructured mesh, the
  seed-point agglomeration of Sec. 3.1.2, macro-edges as chains of finer
  faces with the P^1 coarse space parameterized by arc length, and the
  multigrid of Sec. 3 on those levels.
* ``adjoint``  -- gradient of a misfit with respect to per-element
  log-permeability through the discrete adjoint of the HDG system
  (derived from eqs. HDG and HDG_flux; not in the paper).

Every function here is pinned by ``tests/test_oracle_*.py`` against facts
the paper and the mathematics fix (energy identities, Propositions 1 and
2, polynomial reproduction, convergence rates, direct solves, the
nested-dissection limit, complex-step derivatives).  Functions without
such a pin say "parity unpinned" in their docstring.
"""
from . import refelem, hdg, mg, adjoint, ipdg, rth, unstructured  # noqa: F401
