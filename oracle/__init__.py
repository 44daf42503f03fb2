"""Plain FP64 CPU oracle for MORE-Stress (model-order-reduced thermal stress of
TSV arrays).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or runs
this package: it is used by ``tests/``, by ``__graft_entry__.smoke()`` and by
the ``cpu_baseline`` leg of ``bench.py``.  It shares no code with the HIP
library; both sides only consume the seeded inputs of ``workloads.py``.

Modules
-------
fem     : materials (eq. 2), trilinear hexahedron, unit-cell mesh and assembly
          (eq. 1, 3-7), centroid stress and von Mises.
mor     : Lagrange surface interpolation (eq. 8-10, 16), the lifted local
          problems and the local basis (eq. 11-15), Galerkin projection
          (eq. 17-19).
array   : the global stage: abstract mesh numbering, assembly, Dirichlet
          data, solve (eq. 20) and per-cell reconstruction (Sec. 4.3-4.4);
          plus the full fine-mesh FEM of a whole array for comparison.
plane   : the paper's evaluation (Sec. 5.1): von Mises on a grid of points
          on each block's mid-height plane, normalised MAE and max-norm error.
krylov  : the condition estimate of the preconditioned system of eq. 20 a
          CG solve yields (Ritz values on its Krylov space), and the
          library's two preconditioners (Jacobi, two-level) written out
          densely from their definitions.

Every floating-point quantity is float64.  Solves use SciPy's sparse LU
(a library primitive); no blocking, fusion or reordering is done beyond what
the paper's equations state, so each step can be checked against the paper
by eye.

Parity status: every function is pinned by tests under ``tests/`` that do not
depend on the oracle itself (closed forms, invariants, brute force, and the
values printed in Table 3).  The only unpinned quantity is absolute agreement
with the paper's error and timing figures, which need the paper's mesh and
its commercial reference solver.
"""
