"""FP64 CPU oracle for the MB-SCB one-cell-inversion hot path.

TEST INFRASTRUCTURE ONLY.  This package is a slow, plain, obviously checkable
CPU implementation of what the GPU library computes.  Only the tests, the
smoke check in ``__graft_entry__`` and the CPU-baseline leg of ``bench.py``
may import it.  The product path (the HIP library and its Python binding)
never imports, links or calls anything here, and this package imports nothing
from the product.

Layout (every function cites the passage of the paper it follows):

* ``quadrature``  Gauss-Legendre S_N nodes and weights (Sec. "ONE-CELL
  INVERSION": Gauss-Legendre used throughout; the S_N equation's 1/2 factor
  fixes sum(w) = 2).
* ``problem``     per-cell data derived from a region table.
* ``balance``     the SCB-in-space x MB-in-time balance equations (eq:scb-mb-a
  to eq:scb-mb-d) with the midpoint and upstream closures and the boundary
  conditions, assembled as one global sparse system per time step, and its
  direct solution.  This is the plain definition of the result.
* ``oci``         one-cell inversion, following the OCI subsection: the
  printed A^+, A^-, S and c^+, c^- per cell, one dense LU per region, block
  Jacobi iterations.
* ``si``          source iteration, following the SI subsection: 4x4 solves
  per cell and angle in transport sweeps with a lagged scalar flux.
* ``stopping``    the scalar-flux stopping rule shared by oci and si.
* ``spectral``    brute-force spectral radii of the two iteration operators
  (Fig. 1 trend).
* ``corrector``   the learned iterate corrector's network (1-D convolutions,
  ReLU, mean squared error and its gradient, Adam): textbook definitions; the
  paper has none.

Parity status: every function here is pinned by tests under ``tests/``
(closed forms, invariants, the paper's printed matrices, brute force),
except where a module header says "parity unpinned".
"""
