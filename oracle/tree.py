"""Reference octree (test infrastructure; never imported by the product path).

The paper encloses the scatterers in one cube at level 0, splits every box
into 8 children level by level down to l_max, drops empty boxes, and defines
Children, Parent, Neighbor (boxes sharing a corner, edge or face) and the
far-field list FF(l,q) = Children(Neighbor(Parent(l,q))) minus Neighbor(l,q)
(Sec. 2.2 and Appendix C).  The paper does not fix an encoding; this module
fixes one that the GPU tree must reproduce bit for bit:

* lo_d = min over points of coordinate d; ext = max_d (max_d - lo_d);
  inv = 2^21 / ext (one IEEE division);
* q_d = min(floor((s_d - lo_d) * inv), 2^21 - 1), one IEEE subtraction then
  one IEEE multiplication, no fused multiply-add;
* code = interleave(q_x, q_y, q_z), bit b of q_x to bit 3b, q_y to 3b+1,
  q_z to 3b+2;
* perm = stable ascending sort by (code, point index);
* the level-l key of a point is code >> 3(21 - l); boxes are distinct keys;
  the parent key is key >> 3;
* neighbours: same-level boxes whose integer coordinates differ by at most 1
  in every axis, the box itself included.

Everything is plain NumPy and Python; it is slow and meant to be obviously
right.
"""

import numpy as np

NBITS = 21


def quantize(points: np.ndarray):
    """Return (lo f64[3], ext f64, inv f64, q i64[n,3])."""
    p = np.asarray(points, dtype=np.float64)
    lo = p.min(axis=0)
    hi = p.max(axis=0)
    ext = float(np.max(hi - lo))
    if not ext > 0.0:
        raise ValueError("all points coincide: the bounding cube has zero size")
    inv = np.float64(2.0 ** NBITS) / np.float64(ext)
    diff = p - lo[None, :]          # IEEE subtraction, elementwise
    scaled = diff * inv             # IEEE multiplication, elementwise
    q = np.floor(scaled).astype(np.int64)
    q = np.minimum(q, (1 << NBITS) - 1)
    return lo, ext, float(inv), q


def interleave(q: np.ndarray) -> np.ndarray:
    """Morton code: bit b of q[:,0] -> bit 3b, q[:,1] -> 3b+1, q[:,2] -> 3b+2."""
    code = np.zeros(q.shape[0], dtype=np.uint64)
    for b in range(NBITS):
        for d in range(3):
            bit = (q[:, d].astype(np.uint64) >> np.uint64(b)) & np.uint64(1)
            code |= bit << np.uint64(3 * b + d)
    return code


def deinterleave(key: int, level: int):
    """Integer box coordinates (ix, iy, iz) of a level-`level` key."""
    ix = iy = iz = 0
    for b in range(level):
        ix |= ((key >> (3 * b)) & 1) << b
        iy |= ((key >> (3 * b + 1)) & 1) << b
        iz |= ((key >> (3 * b + 2)) & 1) << b
    return ix, iy, iz


def encode(ix: int, iy: int, iz: int, level: int) -> int:
    key = 0
    for b in range(level):
        key |= ((ix >> b) & 1) << (3 * b)
        key |= ((iy >> b) & 1) << (3 * b + 1)
        key |= ((iz >> b) & 1) << (3 * b + 2)
    return key


class Octree:
    """Reference octree of `depth` levels below the root cube.

    Attributes
    ----------
    codes : u64[n]          Morton codes in user order
    perm : i64[n]           perm[i] = user index of the i-th point in sorted order
    keys[l] : u64[B_l]      sorted distinct keys at level l (l = 0..depth)
    point_box[l] : i64[n]   box index at level l of each sorted point
    parent[l] : i64[B_l]    index of the parent box at level l-1 (l >= 1)
    box_start[l] : i64[B_l+1]  point ranges (sorted order) of the boxes
    nbr[l] : list of sorted int arrays   neighbours (self included)
    ff[l] : list of sorted int arrays    far-field list (l >= 2)
    """

    def __init__(self, points: np.ndarray, depth: int):
        if depth < 0 or depth > NBITS:
            raise ValueError("depth out of range")
        self.depth = depth
        self.lo, self.ext, self.inv, q = quantize(points)
        self.codes = interleave(q)
        n = self.codes.shape[0]
        self.perm = np.lexsort((np.arange(n), self.codes))
        sc = self.codes[self.perm]
        self.keys, self.point_box, self.box_start, self.parent = [], [], [], []
        self.coords = []
        for l in range(depth + 1):
            k = sc >> np.uint64(3 * (NBITS - l))
            first = np.ones(n, dtype=bool)
            first[1:] = k[1:] != k[:-1]
            starts = np.nonzero(first)[0]
            self.keys.append(k[starts])
            self.point_box.append(np.cumsum(first) - 1)
            self.box_start.append(np.concatenate([starts, [n]]).astype(np.int64))
            self.coords.append(np.array([deinterleave(int(x), l) for x in k[starts]], dtype=np.int64).reshape(-1, 3))
            if l == 0:
                self.parent.append(np.full(len(starts), -1, dtype=np.int64))
            else:
                pk = self.keys[l] >> np.uint64(3)
                self.parent.append(np.searchsorted(self.keys[l - 1], pk).astype(np.int64))
        self.nbr = [self._neighbours(l) for l in range(depth + 1)]
        self.ff = [None, None] + [self._far_field(l) for l in range(2, depth + 1)]

    def _neighbours(self, l):
        index = {int(k): i for i, k in enumerate(self.keys[l])}
        out = []
        side = 1 << l
        for (ix, iy, iz) in self.coords[l]:
            lst = []
            for dz in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dx in (-1, 0, 1):
                        jx, jy, jz = ix + dx, iy + dy, iz + dz
                        if 0 <= jx < side and 0 <= jy < side and 0 <= jz < side:
                            j = index.get(encode(jx, jy, jz, l))
                            if j is not None:
                                lst.append(j)
            out.append(np.array(sorted(lst), dtype=np.int64))
        return out

    def _far_field(self, l):
        children = [[] for _ in range(len(self.keys[l - 1]))]
        for i, p in enumerate(self.parent[l]):
            children[p].append(i)
        out = []
        for i in range(len(self.keys[l])):
            near = set(self.nbr[l][i].tolist())
            lst = []
            for pn in self.nbr[l - 1][self.parent[l][i]]:
                for c in children[pn]:
                    if c not in near:
                        lst.append(c)
            out.append(np.array(sorted(lst), dtype=np.int64))
        return out

    def centers(self, l):
        """f64[B_l,3] box centres lo + (q + 1/2) ext / 2^l."""
        h = self.ext / (1 << l)
        return self.lo[None, :] + (self.coords[l] + 0.5) * h
