"""The synthetic meshes are closed, outward-oriented surfaces of the stated size (CPU only)."""

import numpy as np
import pytest

from synthetic import icosphere, nystrom3, split_ring, split_torus, torus


@pytest.mark.parametrize("name", ["sphere", "torus", "split_torus", "split_ring"])
def test_closed_and_outward(name):
    """sum w n = 0 (a closed surface) and the divergence-theorem volume
    sum w (s . n) / 3 equals the body's volume up to the polygon deficit."""
    R, r, gap = 3.5, 1.5, np.pi / 10
    mesh, vol = {
        "sphere": (icosphere(8), 4.0 / 3.0 * np.pi),
        "torus": (torus(R, r, 72, 24), 2 * np.pi * R * np.pi * r * r),
        "split_torus": (split_torus(R, r, gap, 72, 24), (2 * np.pi - gap) * R * np.pi * r * r),
        "split_ring": (split_ring(1.0, 0.2, 0.1, 0.2, h=0.05), (1.0 - 0.6 ** 2) * 0.1 - 0.2 * 0.2 * 0.1),
    }[name]
    q = nystrom3(mesh)
    w, n, s = q["weights"], q["normals"], q["points"]
    assert np.linalg.norm((w[:, None] * n).sum(0)) <= 1e-12 * w.sum()
    v = np.sum(w * np.sum(s * n, 1)) / 3.0
    assert v > 0 and abs(v / vol - 1.0) <= 0.02, (name, v, vol)
