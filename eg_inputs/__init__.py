"""Seeded synthetic inputs shared by the FP64 oracle and the HIP library.

This package holds mesh generators (vertex coordinates, element-to-vertex
connectivity, boundary tags), the seeded draws of the batched workload and
seeded random arrays.  It contains none of the discretisation's arithmetic:
no quadrature, no basis, no geometry factors, no flux.  Both sides derive
everything else from these arrays on their own.
"""

from .meshes import (  # noqa: F401
    TAG_INTERIOR,
    TAG_WALL,
    TAG_FARFIELD,
    TAG_EXACT,
    TAG_SYMMETRY,
    Mesh,
    ogrid,
    cubed_sphere_shell,
    box,
    radial_map,
    wall_bumps,
    reorient,
    mapped,
    clip,
    straight_nodes,
    QUAD9_REF,
    QUAD9_CORNER,
    node_ref,
    node_of_vertex,
)
from .draws import batch_draws, bump_centers, seeded_array  # noqa: F401
from .polymesh import PolyMesh, box_poly, sphere_poly, from_hexes, TET, PRISM, TET_FACES, PRISM_FACES  # noqa: F401
