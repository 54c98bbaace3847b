"""Plain FP64 CPU oracle for the fourth-order cut-cell elliptic solver
(Zhu, Li, Zhang: "A Fast Fourth-Order Cut Cell Method for Solving Elliptic
Equations in Two-Dimensional Irregular Domains").

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package: only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` use it.  It shares no code with the HIP library.

Modules
  geometry        cut cells, Green's-formula cubature, Alg. 1 merging (Sections 2.4, 3.1)
  discretization  regular stencils, R-PLG lattices, weighted least squares,
                  assembly of L and N (Sections 2.2, 2.3, 3.2-3.4)
  multigrid       V-cycle (Alg. 2), SMO-1/SMO-2, transfers, bottom LU,
                  Alg. 3 ordering, transpose solve (Section 4)
  norms           volume-weighted error norms (Section 5)

Parity status of each function is recorded in its docstring; functions
without an independent pin say "parity unpinned": the choice of lattice in
Discretization.lattice_pool / plg, the exact order of alg3_order, and the
depth heuristic Hierarchy.select_depth (the paper fixes none of them).
"""
from .geometry import CutGrid, GeometryError, build_cut_grid  # noqa: F401
try:
    from .discretization import Discretization, PLGError, discretize  # noqa: F401
except ImportError:  # pragma: no cover
    pass
