"""Seeded, synthetic inputs shared by the oracle and the HIP path.

This package holds meshes (connectivity, corner coordinates, curved edges,
boundary tags), analytic initial and boundary data, and the named workload
configurations.  It contains none of the method's arithmetic: no GLL nodes,
no geometry, no operator, no solver, no time stepping.  Node coordinates at
GLL points are computed by each consumer from the corner/arc description.
"""

from .mesh import HexMesh, structured_slice, structured_box, quad_mesh_from_vertices, cylinder_tank_mesh
from . import waves, configs

__all__ = [
    "HexMesh",
    "structured_slice",
    "structured_box",
    "quad_mesh_from_vertices",
    "cylinder_tank_mesh",
    "waves",
    "configs",
]
