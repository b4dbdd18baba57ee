"""Test-case builders: the same seeded workload handed to the oracle and to
the HIP library (tests only)."""
import numpy as np

from workloads import icosphere, box_mesh, random_vector

# quadrature orders shared by both sides in the parity tests (the library's
# defaults); the oracle's own defaults are higher
QUAD = dict(touch_out=6, touch_in=6, close_out=5, close_in=5, far_out=4, far_in=4)

CASES = {
    # name: (mesh builder, eps_r, sigma, freq, grid n, near radius)
    "sphere2": (lambda: icosphere(2), 4.0, 0.0, 150e6, 12, 3),
    "sphere2_lossy": (lambda: icosphere(2), 4.0, 0.5, 150e6, 10, 2),
    "bar_small": (lambda: box_mesh((100e-6, 10e-6, 5e-6), (30, 3, 2)), 1.0, 5.8e7, 10e9, 20, 3),
    # good conductor on a coarse mesh: skin depth 5 um, edges 0.5 mm
    # (|Im k_i| l ~ 140, strong-loss inner integration)
    "box_cond": (lambda: box_mesh((3e-3, 2e-3, 2e-3), (6, 4, 4)), 1.0, 1e7, 1e9, 12, 3),
}


def mesh_of(name):
    return CASES[name][0]()


def gpu_problem(name, quad=QUAD):
    from paper_2003_11679_amd import Problem
    build, eps_r, sigma, freq, n, R = CASES[name]
    xyz, tri = build()
    p = Problem(freq)
    p.add_object(xyz, tri, eps_r=eps_r, sigma=sigma)
    p.set_grid(-1, n=n, near_radius=R)
    p.set_quadrature(**quad)
    p.setup()
    return p


_oracle_cache = {}


def oracle_aim(name, medium, quad=QUAD):
    """Oracle AIM operator of the exterior (medium -1) or interior (0)."""
    key = (name, medium, tuple(sorted(quad.items())))
    if key in _oracle_cache:
        return _oracle_cache[key]
    from oracle.rwg import RWGMesh
    from oracle.aim import Grid, AIMOperator
    from oracle import physics as ph
    build, eps_r, sigma, freq, n, R = CASES[name]
    m = RWGMesh([build()])
    k = ph.wavenumber(freq, 1.0) if medium == -1 else ph.wavenumber(freq, eps_r, 1.0, sigma)
    op = AIMOperator(m, Grid.enclosing(m.xyz, n), k, near_radius=R, rules=quad)
    _oracle_cache[key] = op
    return op


def vec(n, seed, nrhs=None):
    return random_vector(n, seed, nrhs)


# Several objects, each on its own grid: three equal spheres (one grid shape,
# batched together) and a box (a shape of its own), different materials.
MULTI_FREQ = 150e6
MULTI_EXT = (12, 2)          # exterior grid points per axis, near radius
MULTI_INT = (8, 2)           # per-object grids
MULTI_OBJECTS = [
    # (builder, eps_r, sigma)
    (lambda: icosphere(1, 0.25, (0.0, 0.0, 0.0)), 4.0, 0.0),
    (lambda: icosphere(1, 0.25, (0.8, 0.0, 0.0)), 2.5, 0.3),
    (lambda: icosphere(1, 0.25, (0.0, 0.8, 0.0)), 6.0, 1.0),
    (lambda: box_mesh((0.4, 0.3, 0.3), (3, 2, 2), (0.8, 0.8, 0.0)), 3.0, 0.05),
]


def multi_meshes(count=4):
    return [b() for b, _, _ in MULTI_OBJECTS[:count]]


def gpu_multi(count=4, quad=QUAD):
    from paper_2003_11679_amd import Problem
    p = Problem(MULTI_FREQ)
    for b, eps_r, sigma in MULTI_OBJECTS[:count]:
        xyz, tri = b()
        p.add_object(xyz, tri, eps_r=eps_r, sigma=sigma)
    p.set_grid(-1, n=MULTI_EXT[0], near_radius=MULTI_EXT[1])
    for i in range(count):
        p.set_grid(i, n=MULTI_INT[0], near_radius=MULTI_INT[1], share=0)
    p.set_quadrature(**quad)
    p.setup()
    return p


def oracle_multi(count=4, quad=QUAD):
    """Oracle AIM operators: exterior on the whole mesh and its grid; each
    interior on its own object's mesh and grid, with the RWG offset of the
    object in the concatenated numbering."""
    key = ("multi", count, tuple(sorted(quad.items())))
    if key in _oracle_cache:
        return _oracle_cache[key]
    from oracle.rwg import RWGMesh
    from oracle.aim import Grid, AIMOperator
    from oracle import physics as ph
    meshes = multi_meshes(count)
    m = RWGMesh(meshes)
    ext = AIMOperator(m, Grid.enclosing(m.xyz, MULTI_EXT[0]), ph.wavenumber(MULTI_FREQ, 1.0),
                      near_radius=MULTI_EXT[1], rules=quad)
    ints, off = [], 0
    for (b, eps_r, sigma), mesh in zip(MULTI_OBJECTS[:count], meshes):
        mi = RWGMesh([mesh])
        op = AIMOperator(mi, Grid.enclosing(mi.xyz, MULTI_INT[0]), ph.wavenumber(MULTI_FREQ, eps_r, 1.0, sigma),
                         near_radius=MULTI_INT[1], rules=quad)
        ints.append((off, mi.nrwg, op, eps_r, sigma))
        off += mi.nrwg
    _oracle_cache[key] = (m, ext, ints)
    return _oracle_cache[key]
