"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This package only builds inputs: triangle meshes shaped like the paper's
scatterers, their three-point Nystrom nodes (points, normals, weights), seeded
complex densities and plane-wave parameters.  It holds none of the method's
arithmetic (no Green's function, no expansion, no solver).
"""

from .meshes import (  # noqa: F401
    Mesh,
    geodesic_ellipsoid,
    icosphere,
    torus,
    split_ring,
    split_torus,
    nystrom3,
    union,
)
from .draws import (  # noqa: F401
    seed_for,
    complex_normal,
    plane_waves,
)
from .configs import config_mesh, CONFIGS  # noqa: F401
