"""Closed, outward-oriented triangle surface meshes (geometry only).

Every generator returns ``(xyz, tri)`` with ``xyz`` float64 ``[nv, 3]`` and
``tri`` int32 ``[nt, 3]``; triangles are counter-clockwise seen from outside, so
the right-hand normal points out of the enclosed volume.
"""
import numpy as np

_PHI = (1.0 + 5.0 ** 0.5) / 2.0

_ICO_V = np.array([
    [-1, _PHI, 0], [1, _PHI, 0], [-1, -_PHI, 0], [1, -_PHI, 0],
    [0, -1, _PHI], [0, 1, _PHI], [0, -1, -_PHI], [0, 1, -_PHI],
    [_PHI, 0, -1], [_PHI, 0, 1], [-_PHI, 0, -1], [-_PHI, 0, 1],
], dtype=np.float64)

_ICO_F = np.array([
    [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
    [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
    [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
    [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
], dtype=np.int64)


def _orient_outward(xyz, tri):
    """Flip every triangle whose normal points towards the centroid of the
    (star-shaped) surface; used for convex generators only."""
    c = xyz.mean(axis=0)
    a, b, d = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    n = np.cross(b - a, d - a)
    s = np.einsum("ij,ij->i", n, (a + b + d) / 3.0 - c)
    tri = tri.copy()
    flip = s < 0
    tri[flip] = tri[flip][:, [0, 2, 1]]
    return tri


def geodesic_sphere(nu, radius=1.0, center=(0.0, 0.0, 0.0)):
    """Icosahedron with every face split into nu*nu triangles, projected to a
    sphere: 20*nu^2 triangles, 10*nu^2 + 2 vertices."""
    nu = int(nu)
    if nu < 1:
        raise ValueError("nu must be >= 1")
    base = _ICO_V / np.linalg.norm(_ICO_V[0])
    keys = {}
    pts = []

    def vid(face, a, b, c):
        w = {}
        for v, cnt in zip(face, (a, b, c)):
            if cnt:
                w[int(v)] = w.get(int(v), 0) + cnt
        key = tuple(sorted(w.items()))
        if key not in keys:
            keys[key] = len(pts)
            p = sum(base[v] * cnt for v, cnt in w.items()) / nu
            pts.append(p / np.linalg.norm(p))
        return keys[key]

    tris = []
    for face in _ICO_F:
        grid = {}
        for i in range(nu + 1):
            for j in range(nu + 1 - i):
                grid[(i, j)] = vid(face, nu - i - j, i, j)
        for i in range(nu):
            for j in range(nu - i):
                tris.append((grid[(i, j)], grid[(i + 1, j)], grid[(i, j + 1)]))
                if i + j < nu - 1:
                    tris.append((grid[(i + 1, j)], grid[(i + 1, j + 1)], grid[(i, j + 1)]))
    xyz = np.asarray(pts) * radius + np.asarray(center, dtype=np.float64)
    tri = np.asarray(tris, dtype=np.int64)
    tri = _orient_outward(xyz, tri)
    return xyz, tri.astype(np.int32)


def icosphere(level, radius=1.0, center=(0.0, 0.0, 0.0)):
    """Icosahedron subdivided ``level`` times (20*4^level triangles)."""
    return geodesic_sphere(2 ** int(level), radius, center)


def ellipsoid(nu, axes=(1.0, 1.0, 1.0), center=(0.0, 0.0, 0.0)):
    """Geodesic sphere scaled by the semi-axes (convex, so outward orientation
    is preserved by a positive diagonal scaling)."""
    xyz, tri = geodesic_sphere(nu)
    xyz = xyz * np.asarray(axes, dtype=np.float64) + np.asarray(center, dtype=np.float64)
    return xyz, tri


def box_mesh(size, divisions, center=(0.0, 0.0, 0.0)):
    """Structured surface mesh of an axis-aligned box.

    ``size`` = (Lx, Ly, Lz), ``divisions`` = (nx, ny, nz) cells per edge; each
    rectangular cell is split along one fixed diagonal.  Triangle count is
    4*(nx*ny + ny*nz + nz*nx)."""
    L = np.asarray(size, dtype=np.float64)
    nd = [int(d) for d in divisions]
    keys = {}
    pts = []

    def vid(ijk):
        if ijk not in keys:
            keys[ijk] = len(pts)
            pts.append([ijk[a] * L[a] / nd[a] for a in range(3)])
        return keys[ijk]

    tris = []
    for ax in range(3):
        u, v = (ax + 1) % 3, (ax + 2) % 3      # (u, v, ax) is right-handed
        for side in (0, nd[ax]):
            outward = side != 0
            for i in range(nd[u]):
                for j in range(nd[v]):
                    def node(di, dj):
                        ijk = [0, 0, 0]
                        ijk[ax] = side
                        ijk[u] = i + di
                        ijk[v] = j + dj
                        return vid(tuple(ijk))
                    a, b, c, d = node(0, 0), node(1, 0), node(1, 1), node(0, 1)
                    if outward:
                        tris.append((a, b, c))
                        tris.append((a, c, d))
                    else:
                        tris.append((a, c, b))
                        tris.append((a, d, c))
    xyz = np.asarray(pts) - L / 2.0 + np.asarray(center, dtype=np.float64)
    return xyz, np.asarray(tris, dtype=np.int32)


def cube_array(nx, ny, edge, pitch, cells, z=0.0):
    """``nx*ny`` cubes of side ``edge`` on a square lattice of ``pitch`` (centre
    to centre) in the z = ``z`` plane, row-major over (ix, iy); each cube has
    ``cells`` x ``cells`` cells per face.  Returns a list of (xyz, tri)."""
    out = []
    x0 = -(nx - 1) * pitch / 2.0
    y0 = -(ny - 1) * pitch / 2.0
    for ix in range(nx):
        for iy in range(ny):
            c = (x0 + ix * pitch, y0 + iy * pitch, z)
            out.append(box_mesh((edge, edge, edge), (cells, cells, cells), center=c))
    return out


def voxel_mesh(mask, cell, center=(0.0, 0.0, 0.0)):
    """Closed surface of a set of boxes: ``mask`` [nx, ny, nz] bool, cubic or
    rectangular cells of size ``cell`` = (dx, dy, dz); every face between a
    filled cell and an empty one becomes two triangles, outward oriented.
    The filled cells must form a solid whose cells touch through faces only
    (no two cells sharing just an edge or a corner)."""
    m = np.asarray(mask, dtype=bool)
    d = np.asarray(cell, dtype=np.float64)
    pad = np.zeros(tuple(n + 2 for n in m.shape), dtype=bool)
    pad[1:-1, 1:-1, 1:-1] = m
    keys, pts, tris = {}, [], []

    def vid(ijk):
        if ijk not in keys:
            keys[ijk] = len(pts)
            pts.append([ijk[a] * d[a] for a in range(3)])
        return keys[ijk]

    for ax in range(3):
        u, v = (ax + 1) % 3, (ax + 2) % 3          # (u, v, ax) right-handed
        for idx in np.argwhere(m):
            for sgn in (-1, 1):
                nb = idx + 1
                nb[ax] += sgn
                if pad[tuple(nb)]:
                    continue
                face = idx[ax] + (1 if sgn > 0 else 0)

                def node(di, dj):
                    ijk = [0, 0, 0]
                    ijk[ax] = face
                    ijk[u] = idx[u] + di
                    ijk[v] = idx[v] + dj
                    return vid(tuple(int(q) for q in ijk))
                a, b, c, e = node(0, 0), node(1, 0), node(1, 1), node(0, 1)
                if sgn > 0:
                    tris += [(a, b, c), (a, c, e)]
                else:
                    tris += [(a, c, b), (a, e, c)]
    xyz = np.asarray(pts)
    xyz = xyz - 0.5 * (xyz.min(axis=0) + xyz.max(axis=0)) + np.asarray(center, dtype=np.float64)
    return xyz, np.asarray(tris, dtype=np.int32)


def split_ring(side=2e-6, width=0.375e-6, gap=0.25e-6, thickness=0.1e-6, cells=16):
    """Square split-ring resonator: a square ring of outer side ``side`` and
    trace ``width`` with a ``gap`` cut through one side, ``thickness`` thick,
    meshed on a ``cells`` x ``cells`` in-plane raster (one cell through the
    thickness).  Defaults give 812 triangles."""
    h = side / cells
    w = max(1, int(round(width / h)))
    g = max(1, int(round(gap / h)))
    m = np.zeros((cells, cells, 1), dtype=bool)
    m[:w, :, 0] = m[-w:, :, 0] = True
    m[:, :w, 0] = m[:, -w:, 0] = True
    c0 = (cells - g) // 2
    m[c0:c0 + g, :w, 0] = False                    # the gap, through the side y = 0
    return voxel_mesh(m, (h, h, thickness))


def mesh_stats(xyz, tri):
    """Counts and signed enclosed volume (positive for outward orientation)."""
    a, b, c = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    vol = np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0
    e = np.sort(np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]]), axis=1)
    ne = len(np.unique(e, axis=0))
    lens = np.linalg.norm(np.concatenate([b - a, c - b, a - c]), axis=1)
    return {"nv": len(xyz), "nt": len(tri), "ne": ne, "volume": vol,
            "edge_min": lens.min(), "edge_mean": lens.mean(), "edge_max": lens.max()}
