"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This package holds only input generation: coarse tetrahedral meshes (vertex
coordinates + cell connectivity), random nodal fields and closed-form source
functions.  It contains none of the method's arithmetic (no refinement, no
element matrices, no stencils, no multigrid), so both the CPU oracle and the
HIP path can consume its output without sharing any computation.
"""
from .meshes import (reference_tet, kuhn_box, jittered_kuhn_box, slab,
                     batch_problems, BatchProblem)
from .fields import uniform_values, sine_source, sine_solution, smooth_field

__all__ = ["reference_tet", "kuhn_box", "jittered_kuhn_box", "slab",
           "batch_problems", "BatchProblem", "uniform_values", "sine_source",
           "sine_solution", "smooth_field"]
