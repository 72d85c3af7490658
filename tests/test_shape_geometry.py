"""The vertex-to-node rule of the shape gradient (CPU): the same nodes as the
mesh generators' three-node rule, the torch path equal to the numpy path, and
vertex normals of a sphere close to radial."""

import numpy as np
import torch

from paper_1211_7177_amd.shape import nodes_of_mesh, nodes_of_triangles, vertex_normals
from synthetic import icosphere, nystrom3, torus


def test_nodes_of_mesh_equal_the_generator_rule():
    m = torus(1.0, 0.3, 12, 6)
    q = nystrom3(m)
    p = nodes_of_mesh(m.vertices, m.triangles)
    for key in ("points", "normals", "weights", "tri_vertices"):
        assert np.allclose(p[key], q[key], rtol=0, atol=1e-15), key
    assert np.array_equal(p["point_tri"], q["point_tri"])


def test_torch_node_rule_equals_numpy_and_differentiates():
    m = icosphere(3)
    tv = m.vertices[m.triangles]
    ref = nodes_of_triangles(tv)
    V = torch.from_numpy(m.vertices.copy()).requires_grad_(True)
    got = nodes_of_triangles(V[torch.from_numpy(m.triangles.astype(np.int64))])
    for r, g in zip(ref, got):
        assert np.allclose(g.detach().numpy(), r, rtol=0, atol=1e-15)
    # total area = sum of weights; its gradient under a uniform scaling is 2 * area
    area = torch.sum(got[2])
    gV = torch.autograd.grad(area, V)[0].numpy()
    assert abs(np.sum(gV * m.vertices) - 2 * area.item()) <= 1e-12 * area.item()


def test_vertex_normals_of_a_sphere_are_nearly_radial():
    m = icosphere(6)
    N = vertex_normals(m.vertices, m.triangles)
    r = m.vertices / np.linalg.norm(m.vertices, axis=1, keepdims=True)
    assert np.allclose(np.linalg.norm(N, axis=1), 1.0, atol=1e-14)
    assert np.min(np.sum(N * r, axis=1)) >= 1 - 1e-3
