"""Seeded synthetic workloads: triangular meshes and initial cell averages.

This package is the only code shared by the GPU path's tests/benchmarks and the
CPU oracle.  It holds none of the scheme's arithmetic: it builds point sets,
triangulates them, and averages analytic initial conditions over triangles.

Workloads (shapes follow the paper's test section):
  * ``sod_strip``      -- 2D Sod shock tube on a strip (paper Sec. 3.2, table of RP data)
  * ``vortex_square``  -- isentropic vortex on [0,10]^2 (paper Sec. 3.1, eqs. ShuVortIC..rhopressDelta)
  * ``explosion_disk`` -- cylindrical explosion on the unit disk (paper Sec. 3.3, EP1 data)
"""
from .mesh import Mesh, strip_mesh, square_graded_mesh, disk_graded_mesh
from .ic import (cell_average, sod_primitive, vortex_primitive, explosion_primitive,
                 prim_to_cons, sod_case, vortex_case, explosion_case, batched_cases,
                 concat_instances)

__all__ = ["Mesh", "strip_mesh", "square_graded_mesh", "disk_graded_mesh",
           "cell_average", "sod_primitive", "vortex_primitive", "explosion_primitive",
           "prim_to_cons", "sod_case", "vortex_case", "explosion_case", "batched_cases",
           "concat_instances"]
