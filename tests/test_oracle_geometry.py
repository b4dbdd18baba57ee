"""Oracle pins: quadrature, closed-form potentials, RWG topology, the C core."""
import math

import numpy as np
import pytest

from workloads import icosphere, box_mesh, geodesic_sphere, mesh_stats
from oracle.rwg import RWGMesh, MeshError
from oracle.quad import collapsed_gauss, edge_graded, vertex_collapsed, self_fan, points_on
from oracle.static import triangle_potentials
from oracle import mom
from oracle._clib import pair_blocks_c, static_pot_c


def _monomial_exact(a, b):
    # int over the unit right triangle of x^a y^b = a! b! / (a+b+2)!, times 2 (area-normalised)
    return 2.0 * math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)


@pytest.mark.parametrize("n", [2, 3, 5, 8])
def test_collapsed_gauss_exact_to_degree_2n_minus_2(n):
    b, w = collapsed_gauss(n)
    for a in range(2 * n - 1):
        for c in range(2 * n - 1 - a):
            got = np.sum(w * b[:, 1] ** a * b[:, 2] ** c)
            assert abs(got - _monomial_exact(a, c)) < 1e-14


@pytest.mark.parametrize("rule", [lambda: edge_graded(10, 1), lambda: vertex_collapsed(10, 2),
                                  lambda: self_fan(10)])
def test_singular_rules_integrate_polynomials(rule):
    b, w = rule()
    assert abs(w.sum() - 1.0) < 1e-14
    for a in range(5):
        for c in range(5 - a):
            assert abs(np.sum(w * b[:, 1] ** a * b[:, 2] ** c) - _monomial_exact(a, c)) < 1e-12


def test_static_potentials_far_point_vs_quadrature():
    rng = np.random.default_rng(3)
    v = rng.standard_normal((1, 3, 3))
    b, w = collapsed_gauss(40)
    P = points_on(v, b)[0]
    A = 0.5 * np.linalg.norm(np.cross(v[0, 1] - v[0, 0], v[0, 2] - v[0, 0]))
    n = np.cross(v[0, 1] - v[0, 0], v[0, 2] - v[0, 0]); n /= np.linalg.norm(n)
    for r in (v[0].mean(0) + 4 * n, v[0].mean(0) + np.array([5.0, -3.0, 1.0])):
        R = np.linalg.norm(P - r, axis=1)
        rho = r - np.dot(r - v[0, 0], n) * n
        I, Ir, g = triangle_potentials(v, r[None, None, :])
        assert abs(I[0, 0] - np.sum(w * A / R)) < 1e-13
        assert np.abs(Ir[0, 0] - ((w * A / R)[:, None] * (P - rho)).sum(0)).max() < 1e-13
        assert np.abs(g[0, 0] - ((w * A / R ** 3)[:, None] * (P - r)).sum(0)).max() < 1e-13


def test_static_gradient_is_gradient_of_potential():
    rng = np.random.default_rng(4)
    v = rng.standard_normal((1, 3, 3))
    c = v[0].mean(0)
    n = np.cross(v[0, 1] - v[0, 0], v[0, 2] - v[0, 0]); n /= np.linalg.norm(n)
    for r in (c + 1e-2 * n, c - 0.3 * n + 0.1 * (v[0, 1] - c), v[0, 0] + 0.2 * (v[0, 0] - c)):
        _, _, g = triangle_potentials(v, r[None, None, :])
        h = 1e-6
        fd = [(triangle_potentials(v, (r + h * e)[None, None, :])[0]
               - triangle_potentials(v, (r - h * e)[None, None, :])[0])[0, 0] / (2 * h)
              for e in np.eye(3)]
        assert np.abs(np.array(fd) - g[0, 0]).max() < 1e-8


def test_static_c_matches_numpy():
    rng = np.random.default_rng(5)
    for _ in range(5):
        v = rng.standard_normal((3, 3)); r = rng.standard_normal(3)
        I, Ir, g = triangle_potentials(v[None], r[None, None, :])
        I2, Ir2, g2 = static_pot_c(v, r)
        assert abs(I[0, 0] - I2) < 1e-13 and np.abs(Ir[0, 0] - Ir2).max() < 1e-13
        assert np.abs(g[0, 0] - g2).max() < 1e-13


def test_pair_blocks_c_matches_numpy():
    m = RWGMesh([icosphere(1)])
    T = len(m.tri)
    tl = np.repeat(np.arange(3), T); sl = np.tile(np.arange(T), 3)
    k = 2.0 - 0.4j
    a1, p1, k1 = mom.pair_blocks_np(m, k, tl, sl, 4, 5)
    a2, p2, k2 = pair_blocks_c(m, k, tl, sl, collapsed_gauss(4), collapsed_gauss(5))
    for x, y in ((a1, a2), (p1, p2), (k1, k2)):
        assert np.abs(x - y).max() <= 1e-12 * np.abs(x).max()


def test_mesh_topology_invariants():
    for xyz, tri in (icosphere(2), box_mesh((3.0, 2.0, 1.0), (6, 4, 2)), geodesic_sphere(5)):
        m = RWGMesh([(xyz, tri)])
        st = mesh_stats(xyz, tri)
        assert st["nv"] - m.nrwg + st["nt"] == 2           # Euler, sphere topology
        assert m.nrwg * 2 == 3 * st["nt"]
        assert st["volume"] > 0
        # every RWG: T+ and T- distinct, opposite signs, total divergence zero
        assert np.all(m.tp != m.tm)
        div_plus = m.length / m.area[m.tp] * m.area[m.tp]
        div_minus = -m.length / m.area[m.tm] * m.area[m.tm]
        assert np.allclose(div_plus + div_minus, 0.0)
        # edge vertex order: a < b and T+ runs a -> b
        assert np.all(m.edge_v[:, 0] < m.edge_v[:, 1])


def test_open_or_flipped_mesh_rejected():
    xyz, tri = icosphere(1)
    with pytest.raises(MeshError):
        RWGMesh([(xyz, tri[1:])])
    bad = tri.copy(); bad[0] = bad[0][[0, 2, 1]]
    with pytest.raises(MeshError):
        RWGMesh([(xyz, bad)])
