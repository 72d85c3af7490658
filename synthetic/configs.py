"""The five benchmark workloads as mesh recipes plus their physical constants.

Shapes and sizes: a dielectric sphere (the paper's Mie benchmark, Sec. 3.2),
a torus and a split ring (the paper's plasmonic examples, Sec. 4.1, Fig. 2),
an ellipsoid, and a large prolate ellipsoid.  The permittivities are fixed
numbers rather than the paper's dispersive models; the host medium is vacuum
(relative eps = mu = 1) and every scatterer has mu = 1.
"""

import numpy as np

from .meshes import geodesic_ellipsoid, icosphere, split_ring, torus

CONFIGS = {
    # sphere a = 1, eps = 2.25, host k0 = 1: 1280 triangles, 3840 points
    1: dict(name="sphere_1280", k0=1.0, eps=2.25, depth=3),
    # torus R = 1, r = 0.3, 200 x 50 x 2 = 20000 triangles, 60000 points, k0 R = 4
    2: dict(name="torus_20k", k0=4.0, eps=complex(-15.0, 1.0), depth=5),
    # batched meshes (ellipsoid, torus, sphere)
    31: dict(name="ellipsoid_8k", k0=2.0, eps=2.25, depth=5),
    32: dict(name="torus_30k", k0=5.0, eps=complex(-15.0, 1.0), depth=5),
    33: dict(name="sphere_81920", k0=10.0, eps=2.25, depth=6),
    # split ring, side 1, width 0.2, thickness 0.1, gap 0.2: 49,404 triangles (148,212 points), k0 = pi/2
    4: dict(name="srr_50k", k0=np.pi / 2, eps=complex(-15.0, 1.0), depth=6),
    # prolate ellipsoid 4:1:1, 1003520 triangles, k0 = 40
    5: dict(name="prolate_1M", k0=40.0, eps=complex(-1e4, 1e2), depth=8),
}


def config_mesh(cfg: int):
    if cfg == 1:
        return icosphere(8, 1.0)
    if cfg == 2:
        return torus(1.0, 0.3, 200, 50)
    if cfg == 31:
        return geodesic_ellipsoid((1.5, 1.0, 0.75), 20)
    if cfg == 32:
        return torus(1.0, 0.3, 250, 60)
    if cfg == 33:
        return icosphere(64, 1.0)
    if cfg == 4:
        return split_ring(1.0, 0.2, 0.1, 0.2, h=0.0087)
    if cfg == 5:
        return geodesic_ellipsoid((4.0, 1.0, 1.0), 224)
    raise KeyError(cfg)
