"""CPU oracle for the matrix-free P1 hot path -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct NumPy/SciPy code that recomputes what the GPU
library computes, straight from the paper's definitions:

* ``refine``  -- explicit recursive regular refinement of each macro-cell with
  the eight children of eq. (bey) (Section 3.1), micro-vertex identification by
  integer barycentric keys, micro-primitive bookkeeping;
* ``fem``     -- element-by-element assembly of the P1 stiffness matrix
  (Section 5.2.1: a_ij is the sum over elements of the integral of
  grad(phi_i).grad(phi_j)), Dirichlet boundary, lumped mass;
* ``mg``      -- nested P1 prolongation from refinement bookkeeping, its
  transpose as restriction, weighted Jacobi, residual, textbook V-cycle with a
  dense Cholesky coarse solve, and the solve loop;
* ``rows``    -- single-row assembly at one micro-vertex by recursive descent
  through the refinement, for sampled checks at levels too large to assemble;
* ``p2``      -- P2 (vertex + edge DoFs, Section 5.1) element matrices by exact
  quadrature, assembly on the explicit micro-mesh with nodes keyed as the
  next level's micro-vertices, and its single-row variant.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never imports, links or
calls it, and it shares no code with the GPU library: the two meet only in the
seeded input generators of ``workloads/``.
"""
