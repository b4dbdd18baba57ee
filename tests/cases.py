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
