"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package only builds workloads: hexahedral meshes stored as face lists,
face coefficients, liquid-fraction fields, right-hand sides, intermediate
velocities and material properties.  It holds
none of the solver's arithmetic (no masking, assembly, aggregation or Krylov
step); those live separately in the oracle and in the HIP library.
"""
from .alloy import al_alloy, al_si_alloy
from .mesh import HexMesh, box_mesh, plate_with_ribs_mesh, concat_meshes, face_coeff
from .fields import (
    fl_linear_x,
    fl_planar_front,
    fl_growing_front,
    rhs_uniform,
    batch_samples,
    uq_front_fl,
    rhs_smooth_series,
    ustar_smooth_series,
    latin_hypercube,
    mlp_initial_weights,
    t_wall_layer,
)

__all__ = [
    "al_alloy",
    "al_si_alloy",
    "HexMesh",
    "box_mesh",
    "plate_with_ribs_mesh",
    "concat_meshes",
    "face_coeff",
    "fl_linear_x",
    "fl_planar_front",
    "fl_growing_front",
    "rhs_uniform",
    "batch_samples",
    "uq_front_fl",
    "rhs_smooth_series",
    "ustar_smooth_series",
    "latin_hypercube",
    "mlp_initial_weights",
    "t_wall_layer",
]
