"""Seeded synthetic inputs shared by the oracle-side tests and the GPU path.

This module only lays out geometry (vertex coordinates and connectivity) and
draws seeded random vectors.  It holds none of the method's arithmetic: no
frames, no influence coefficients, no tree, no solver.  Both the CPU oracle
and the HIP library receive the arrays produced here unchanged.

Conventions (shared with both sides, stated once here):
  * vertices ``xyz`` float64 [nv, 3] in metres, global frame;
  * ``conn`` int64 [ne, 3] (triangles) or [ne, 4] (planar rectangles),
    0-based, counter-clockwise about the intended element normal, with the
    first edge v0->v1 along the intended first in-plane axis s1;
  * DD and traction vectors float64, element-major, [s1, s2, n] per element.
"""
from .meshes import (  # noqa: F401
    Mesh,
    rect_grid,
    square_fault,
    disk_mesh,
    rect_tri_mesh,
    three_disks,
    hf_fault_mesh,
    batched_faults,
    rhs_columns,
    penny_active_mask,
    gaussian_pressure_traction,
    tangent_state,
    tangent_rhs,
)
