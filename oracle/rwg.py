"""RWG basis functions on closed oriented triangle meshes (Sec. III-A).

The paper expands n x E and n x H in RWG functions (Rao-Wilton-Glisson, 1982)
and tests with them; it only cites the definition, so the standard one is used:
on the triangle T+ of edge n, f_n(r) = l_n/(2 A+) (r - p+); on T-,
f_n(r) = -l_n/(2 A-) (r - p-), with p+/- the vertices opposite the edge, and
div f_n = +l_n/A+ on T+, -l_n/A- on T-.

Numbering convention (an interface shared with the library, so results can be
compared index by index): RWG functions are the interior edges {a, b}, a < b
(global vertex indices after objects are concatenated), sorted by (a, b); T+ is
the triangle whose counter-clockwise vertex order runs a -> b.
"""
import numpy as np


class MeshError(ValueError):
    pass


class RWGMesh:
    """Concatenated objects with RWG topology and per-triangle geometry."""

    def __init__(self, objects):
        xyz_l, tri_l, obj_of_tri = [], [], []
        off = 0
        for i, (xyz, tri) in enumerate(objects):
            xyz = np.asarray(xyz, dtype=np.float64)
            tri = np.asarray(tri, dtype=np.int64)
            xyz_l.append(xyz)
            tri_l.append(tri + off)
            obj_of_tri.append(np.full(len(tri), i, dtype=np.int64))
            off += len(xyz)
        self.xyz = np.concatenate(xyz_l)
        self.tri = np.concatenate(tri_l)
        self.tri_obj = np.concatenate(obj_of_tri)
        self.nobj = len(objects)
        self._geometry()
        self._topology()

    def _geometry(self):
        v = self.xyz[self.tri]                      # [T,3,3]
        cr = np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0])
        nrm = np.linalg.norm(cr, axis=1)
        if np.any(nrm <= 0):
            raise MeshError("degenerate triangle")
        self.area = 0.5 * nrm
        self.normal = cr / nrm[:, None]
        self.verts = v
        self.centroid = ((v[:, 0] + v[:, 1]) + v[:, 2]) / 3.0

    def _topology(self):
        T = len(self.tri)
        d = {}
        for t in range(T):
            for e in range(3):
                a, b = int(self.tri[t, (e + 1) % 3]), int(self.tri[t, (e + 2) % 3])
                key = (min(a, b), max(a, b))
                d.setdefault(key, []).append((t, e, a < b))
        keys = sorted(d.keys())
        E = len(keys)
        tp = np.empty(E, np.int64); tm = np.empty(E, np.int64)
        ep = np.empty(E, np.int64); em = np.empty(E, np.int64)
        tri_rwg = np.full((T, 3), -1, np.int64)
        tri_sign = np.zeros((T, 3), np.float64)
        for n, key in enumerate(keys):
            lst = d[key]
            if len(lst) != 2:
                raise MeshError(f"edge {key} has {len(lst)} triangles (mesh not closed 2-manifold)")
            (t1, e1, f1), (t2, e2, f2) = lst
            if f1 == f2:
                raise MeshError(f"edge {key}: inconsistent orientation")
            if not f1:
                (t1, e1, f1), (t2, e2, f2) = (t2, e2, f2), (t1, e1, f1)
            tp[n], ep[n], tm[n], em[n] = t1, e1, t2, e2
            tri_rwg[t1, e1] = n; tri_sign[t1, e1] = 1.0
            tri_rwg[t2, e2] = n; tri_sign[t2, e2] = -1.0
        self.nrwg = E
        self.edge_v = np.asarray(keys, dtype=np.int64)
        self.tp, self.tm, self.ep, self.em = tp, tm, ep, em
        self.length = np.linalg.norm(self.xyz[self.edge_v[:, 1]] - self.xyz[self.edge_v[:, 0]], axis=1)
        self.tri_rwg = tri_rwg
        self.tri_sign = tri_sign
        self.rwg_obj = self.tri_obj[tp]
        # per (triangle, local edge): length and free vertex
        self.tri_len = self.length[tri_rwg]
        self.tri_free = self.verts                     # free vertex of local edge e is vertex e

    def basis_on_triangle(self, t, pts):
        """f for the three local edges of triangle t at points pts [...,3]:
        returns vals [...,3(edge),3(xyz)] and divergences [3]."""
        s = self.tri_sign[t]
        l = self.tri_len[t]
        A = self.area[t]
        coef = s * l / (2.0 * A)
        vals = coef[None, :, None] * (pts[:, None, :] - self.verts[t][None, :, :])
        div = s * l / A
        return vals, div

    def obj_rwg_range(self, i):
        idx = np.nonzero(self.rwg_obj == i)[0]
        return idx[0], idx[-1] + 1
