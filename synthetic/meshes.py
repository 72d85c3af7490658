"""Planar triangle meshes of the paper's scatterer shapes and their Nystrom nodes.

The paper discretises every surface into flat triangles (Sec. 2.2, Fig. 2) and
takes the unit normal of a triangle ABC as AB x AC / |AB x AC| (Appendix B,
eq. B.1).  Every mesh built here orders its triangles counter-clockwise seen
from outside, so that this normal points out of the scatterer.

`nystrom3` places three quadrature nodes in each triangle at barycentric
coordinates (2/3, 1/6, 1/6) and permutations, each with weight area/3 (the
degree-2 interior rule).  With one node at the centroid and weight = area it
would be the paper's own rule (eq. 2.8 and the text after it).
"""

from dataclasses import dataclass

import numpy as np


@dataclass
class Mesh:
    """A closed triangle mesh: vertices f64[nv,3], triangles i32[nt,3] (CCW from outside)."""

    vertices: np.ndarray
    triangles: np.ndarray

    @property
    def ntri(self) -> int:
        return int(self.triangles.shape[0])

    def tri_vertices(self) -> np.ndarray:
        """f64[nt,3,3]: the three corner positions of every triangle."""
        return np.ascontiguousarray(self.vertices[self.triangles], dtype=np.float64)


def _dedupe(points: np.ndarray, tris: np.ndarray, tol: float = 1e-11):
    key = np.round(points / tol).astype(np.int64)
    _, first, inv = np.unique(key, axis=0, return_index=True, return_inverse=True)
    inv = inv.reshape(-1)
    return points[first], inv[tris].astype(np.int32)


_ICO_V = None


def _icosahedron():
    t = (1.0 + 5.0 ** 0.5) / 2.0
    v = np.array(
        [
            [-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
            [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
            [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1],
        ],
        dtype=np.float64,
    )
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array(
        [
            [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
            [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
            [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
            [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
        ],
        dtype=np.int64,
    )
    return v, f


def _geodesic_unit_sphere(nu: int):
    """Frequency-nu geodesic sphere: each icosahedron face split into nu^2
    triangles on a barycentric grid, every grid point projected radially."""
    v, f = _icosahedron()
    # barycentric grid indices (i, j) with i + j <= nu; point = A + (B-A) i/nu + (C-A) j/nu
    pts = []
    tris = []
    base = 0
    idx = {}
    for i in range(nu + 1):
        for j in range(nu + 1 - i):
            idx[(i, j)] = len(idx)
    nloc = len(idx)
    loc_tris = []
    for i in range(nu):
        for j in range(nu - i):
            a = idx[(i, j)]
            b = idx[(i + 1, j)]
            c = idx[(i, j + 1)]
            loc_tris.append((a, b, c))
            if i + j < nu - 1:
                d = idx[(i + 1, j + 1)]
                loc_tris.append((b, d, c))
    loc_tris = np.array(loc_tris, dtype=np.int64)
    ij = np.array(list(idx.keys()), dtype=np.float64) / nu
    for (ia, ib, ic) in f:
        A, B, C = v[ia], v[ib], v[ic]
        p = A[None, :] + ij[:, :1] * (B - A)[None, :] + ij[:, 1:2] * (C - A)[None, :]
        p /= np.linalg.norm(p, axis=1, keepdims=True)
        pts.append(p)
        tris.append(loc_tris + base)
        base += nloc
    pts = np.concatenate(pts)
    tris = np.concatenate(tris)
    return _dedupe(pts, tris)


def geodesic_ellipsoid(axes, nu: int) -> Mesh:
    """Geodesic ellipsoid with semi-axes `axes`: 20*nu^2 triangles."""
    p, t = _geodesic_unit_sphere(nu)
    p = p * np.asarray(axes, dtype=np.float64)[None, :]
    return _orient_outward(Mesh(p, t), center=np.zeros(3))


def icosphere(nu: int, radius: float = 1.0) -> Mesh:
    """Geodesic sphere of the given radius with 20*nu^2 triangles (nu = 8 gives 1280)."""
    return geodesic_ellipsoid((radius, radius, radius), nu)


def torus(R: float, r: float, nu: int, nv: int) -> Mesh:
    """Parametric torus about the z axis: nu x nv quads, 2*nu*nv triangles."""
    u = 2.0 * np.pi * np.arange(nu) / nu
    v = 2.0 * np.pi * np.arange(nv) / nv
    U, V = np.meshgrid(u, v, indexing="ij")
    X = (R + r * np.cos(V)) * np.cos(U)
    Y = (R + r * np.cos(V)) * np.sin(U)
    Z = r * np.sin(V)
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    I, J = np.meshgrid(np.arange(nu), np.arange(nv), indexing="ij")
    I = I.ravel()
    J = J.ravel()
    a = I * nv + J
    b = ((I + 1) % nu) * nv + J
    c = ((I + 1) % nu) * nv + (J + 1) % nv
    d = I * nv + (J + 1) % nv
    tris = np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, d], 1)]).astype(np.int32)
    mesh = Mesh(pts, tris)
    # outward test against the nearest point of the tube's centre circle
    cen = mesh.vertices[mesh.triangles].mean(axis=1)
    rho = np.hypot(cen[:, 0], cen[:, 1])
    core = np.stack([R * cen[:, 0] / rho, R * cen[:, 1] / rho, np.zeros_like(rho)], 1)
    return _orient_by_reference(mesh, core)


def split_torus(R: float, r: float, gap: float, nu: int, nv: int, nc: int = 4) -> Mesh:
    """Torus about the z axis (major radius R, tube radius r) with the sector
    |phi| < gap/2 around +x removed, closed by two flat discs: nu segments along
    the remaining angle, nv around the tube, nc rings on each disc (the outer
    ring is the tube's end ring, so the surface is conforming)."""
    phis = gap / 2.0 + (2.0 * np.pi - gap) * np.arange(nu + 1) / nu
    v = 2.0 * np.pi * np.arange(nv) / nv
    U, V = np.meshgrid(phis, v, indexing="ij")
    pts = [np.stack([((R + r * np.cos(V)) * np.cos(U)).ravel(), ((R + r * np.cos(V)) * np.sin(U)).ravel(),
                     (r * np.sin(V)).ravel()], axis=1)]
    I, J = np.meshgrid(np.arange(nu), np.arange(nv), indexing="ij")
    I, J = I.ravel(), J.ravel()
    a, b = I * nv + J, (I + 1) * nv + J
    c, d = (I + 1) * nv + (J + 1) % nv, I * nv + (J + 1) % nv
    tris = [np.stack([a, b, c], 1), np.stack([a, c, d], 1)]
    ref = []                                    # outward reference point per triangle (a point inside)
    base = (nu + 1) * nv
    for end, phi in ((0, phis[0]), (nu, phis[-1])):
        cen = np.array([R * np.cos(phi), R * np.sin(phi), 0.0])
        rings = []
        for k in range(1, nc):                  # inner rings of the disc, then the tube's end ring
            rr = r * k / nc
            ring = np.stack([(R + rr * np.cos(v)) * np.cos(phi), (R + rr * np.cos(v)) * np.sin(phi), rr * np.sin(v)], 1)
            pts.append(ring)
            rings.append(base + np.arange(nv))
            base += nv
        pts.append(cen[None, :])
        ci = base
        base += 1
        rings.append(end * nv + np.arange(nv))
        jn = (np.arange(nv) + 1) % nv
        tris.append(np.stack([np.full(nv, ci), rings[0], rings[0][jn]], 1))
        for k in range(len(rings) - 1):
            p0, p1 = rings[k], rings[k + 1]
            tris.append(np.stack([p0, p1, p1[jn]], 1))
            tris.append(np.stack([p0, p1[jn], p0[jn]], 1))
        # the disc's outward side is away from the remaining tube, i.e. into the gap
        t_phi = np.array([-np.sin(phi), np.cos(phi), 0.0]) * (-1.0 if end == 0 else 1.0)
        ref.append((cen, t_phi))
    mesh = Mesh(np.concatenate(pts), np.concatenate(tris).astype(np.int32))
    tv = mesh.tri_vertices()
    nrm = np.cross(tv[:, 1] - tv[:, 0], tv[:, 2] - tv[:, 0])
    cent = tv.mean(axis=1)
    ntube = 2 * nu * nv
    rho = np.hypot(cent[:ntube, 0], cent[:ntube, 1])
    core = np.stack([R * cent[:ntube, 0] / rho, R * cent[:ntube, 1] / rho, np.zeros(ntube)], 1)
    out = np.empty_like(cent)
    out[:ntube] = cent[:ntube] - core
    ncap = (len(cent) - ntube) // 2
    out[ntube:ntube + ncap] = ref[0][1]
    out[ntube + ncap:] = ref[1][1]
    flip = np.einsum("ij,ij->i", nrm, out) < 0
    t = mesh.triangles.copy()
    t[flip] = t[flip][:, [0, 2, 1]]
    return Mesh(mesh.vertices, t.astype(np.int32))


def split_ring(side: float = 1.0, width: float = 0.2, thickness: float = 0.1,
               gap: float = 0.2, h: float = 0.02) -> Mesh:
    """Square split ring in the xy plane, centred at the origin, the gap cut
    through the middle of the +x side.  Built as a closed polyhedral surface of
    axis-aligned rectangles, each rectangle gridded at spacing ~h."""
    s = side / 2.0
    w = width
    zt = thickness / 2.0
    g = gap / 2.0
    # The ring is the union of boxes; describe its outline in the xy plane as a
    # polygon and extrude.  Outer square [-s,s]^2, inner [-s+w, s-w]^2, minus the
    # gap strip |y| < g on the +x side (x in [s-w, s]).
    outer = [(-s, -s), (s, -s), (s, -g), (s - w, -g), (s - w, -s + w), (-s + w, -s + w),
             (-s + w, s - w), (s - w, s - w), (s - w, g), (s, g), (s, s), (-s, s)]
    # The polygon above traces the C-shaped outline counter-clockwise.
    poly = np.array(outer, dtype=np.float64)
    tris = []
    pts = []

    def add_rect(p0, e1, e2):
        n1 = max(1, int(np.ceil(np.linalg.norm(e1) / h)))
        n2 = max(1, int(np.ceil(np.linalg.norm(e2) / h)))
        a = np.arange(n1 + 1) / n1
        b = np.arange(n2 + 1) / n2
        A, B = np.meshgrid(a, b, indexing="ij")
        P = p0[None, None, :] + A[..., None] * e1[None, None, :] + B[..., None] * e2[None, None, :]
        base = sum(len(q) for q in pts)
        pts.append(P.reshape(-1, 3))
        I, J = np.meshgrid(np.arange(n1), np.arange(n2), indexing="ij")
        I = I.ravel()
        J = J.ravel()
        q00 = base + I * (n2 + 1) + J
        q10 = base + (I + 1) * (n2 + 1) + J
        q11 = base + (I + 1) * (n2 + 1) + J + 1
        q01 = base + I * (n2 + 1) + J + 1
        tris.append(np.stack([q00, q10, q11], 1))
        tris.append(np.stack([q00, q11, q01], 1))

    # side walls: one rectangle per polygon edge
    m = len(poly)
    for i in range(m):
        p0 = np.array([poly[i][0], poly[i][1], -zt])
        p1 = np.array([poly[(i + 1) % m][0], poly[(i + 1) % m][1], -zt])
        add_rect(p0, p1 - p0, np.array([0.0, 0.0, 2 * zt]))
    # top and bottom faces: the C shape as a union of 5 axis-aligned rectangles
    rects = [
        (-s, -s, 2 * s, w),              # bottom bar
        (-s, s - w, 2 * s, w),           # top bar
        (-s, -s + w, w, 2 * s - 2 * w),  # left bar
        (s - w, -s + w, w, s - w - g),   # lower right stub
        (s - w, g, w, s - w - g),        # upper right stub
    ]
    for (x0, y0, dx, dy) in rects:
        add_rect(np.array([x0, y0, zt]), np.array([dx, 0, 0.0]), np.array([0, dy, 0.0]))
        add_rect(np.array([x0, y0, -zt]), np.array([dx, 0, 0.0]), np.array([0, dy, 0.0]))
    P = np.concatenate(pts)
    T = np.concatenate(tris)
    mesh = Mesh(P, T.astype(np.int32))
    return _orient_split_ring(mesh, poly, zt)


def _normals_raw(mesh: Mesh):
    tv = mesh.tri_vertices()
    return np.cross(tv[:, 1] - tv[:, 0], tv[:, 2] - tv[:, 0]), tv.mean(axis=1)


def _orient_outward(mesh: Mesh, center) -> Mesh:
    nrm, cen = _normals_raw(mesh)
    flip = np.einsum("ij,ij->i", nrm, cen - center[None, :]) < 0
    t = mesh.triangles.copy()
    t[flip] = t[flip][:, [0, 2, 1]]
    return Mesh(mesh.vertices, t.astype(np.int32))


def _orient_by_reference(mesh: Mesh, inner_points) -> Mesh:
    nrm, cen = _normals_raw(mesh)
    flip = np.einsum("ij,ij->i", nrm, cen - inner_points) < 0
    t = mesh.triangles.copy()
    t[flip] = t[flip][:, [0, 2, 1]]
    return Mesh(mesh.vertices, t.astype(np.int32))


def _point_in_poly(x, y, poly):
    inside = np.zeros(x.shape, dtype=bool)
    m = len(poly)
    for i in range(m):
        x0, y0 = poly[i]
        x1, y1 = poly[(i + 1) % m]
        cond = (y0 > y) != (y1 > y)
        xi = x0 + (y - y0) * (x1 - x0) / np.where(y1 != y0, y1 - y0, 1.0)
        inside ^= cond & (x < xi)
    return inside


def _orient_split_ring(mesh: Mesh, poly, zt) -> Mesh:
    nrm, cen = _normals_raw(mesh)
    unit = nrm / np.linalg.norm(nrm, axis=1, keepdims=True)
    probe = cen + 1e-6 * unit
    inside = _point_in_poly(probe[:, 0], probe[:, 1], poly) & (np.abs(probe[:, 2]) < zt)
    t = mesh.triangles.copy()
    t[inside] = t[inside][:, [0, 2, 1]]
    return Mesh(mesh.vertices, t.astype(np.int32))


_BARY3 = np.array([[2.0 / 3, 1.0 / 6, 1.0 / 6],
                   [1.0 / 6, 2.0 / 3, 1.0 / 6],
                   [1.0 / 6, 1.0 / 6, 2.0 / 3]])


def nystrom3(mesh: Mesh):
    """Three-node interior rule on every triangle.

    Returns dict with points f64[3nt,3], normals f64[3nt,3] (the face normal
    AB x AC normalised, eq. B.1), weights f64[3nt] (area/3), point_tri i32[3nt]
    (point 3*t + i lies in triangle t) and tri_vertices f64[nt,3,3].
    """
    tv = mesh.tri_vertices()
    cr = np.cross(tv[:, 1] - tv[:, 0], tv[:, 2] - tv[:, 0])
    area2 = np.linalg.norm(cr, axis=1)
    nrm = cr / area2[:, None]
    pts = np.einsum("qk,tkd->tqd", _BARY3, tv).reshape(-1, 3)
    normals = np.repeat(nrm, 3, axis=0)
    weights = np.repeat(area2 / 6.0, 3)
    point_tri = np.repeat(np.arange(mesh.ntri, dtype=np.int32), 3)
    return {
        "points": np.ascontiguousarray(pts),
        "normals": np.ascontiguousarray(normals),
        "weights": np.ascontiguousarray(weights),
        "point_tri": point_tri,
        "tri_vertices": tv,
    }


def union(meshes, offsets):
    """Several closed meshes as one triangle set, mesh i translated by offsets[i].
    Returns (mesh, tri_region) with tri_region[t] = index of the mesh holding triangle t."""
    verts, tris, reg = [], [], []
    base = 0
    for i, (m, off) in enumerate(zip(meshes, offsets)):
        verts.append(m.vertices + np.asarray(off, dtype=np.float64)[None, :])
        tris.append(m.triangles + base)
        reg.append(np.full(len(m.triangles), i, dtype=np.int32))
        base += len(m.vertices)
    return Mesh(np.concatenate(verts), np.concatenate(tris).astype(np.int32)), np.concatenate(reg)
