"""Seeded synthetic inputs shared by the HIP path's tests/benchmark and the CPU oracle.

This package holds input data only: simplicial meshes of the unit square / unit cube,
vertex jitter, per-element material coefficients, polynomial degrees, point-source
locations and Neumann tags of box faces.  It contains none of the discretisation's arithmetic (no basis, quadrature,
local matrices or solves), so that the oracle and the GPU library stay independent.
"""
from .rhs import random_vector  # noqa: F401
from .meshes import (  # noqa: F401
    Problem,
    unit_square_tris,
    kuhn_cube_tets,
    five_tet_box,
    jitter_vertices,
    make_problem,
    tag_box_faces,
    CONFIGS,
)
