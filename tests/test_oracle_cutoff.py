"""Oracle pins of the local forms of the AIM operator: the small-object
bypass (Sec. III-D-2 item b: every pair near, so the grid part equals the
precorrection and the operator is the direct one) and the five-skin-depth
cutoff (Sec. V), both against the dense Galerkin operators."""
import numpy as np
import pytest

from workloads import icosphere, box_mesh, random_vector
from oracle.rwg import RWGMesh
from oracle.aim import Grid, AIMOperator
from oracle.mom import dense_operators, L_from
from oracle import physics as ph
from cases import QUAD


def _dense(m, k):
    A, P, K = dense_operators(m, k, rules=QUAD)
    return L_from(A, P, k), K


def test_all_near_bypass_equals_dense_and_grid_form():
    m = RWGMesh([icosphere(1)])
    k = ph.wavenumber(150e6, 4.0, 1.0, 0.2)
    g = Grid.enclosing(m.xyz, 8)
    a = AIMOperator(m, g, k, near_radius=6, rules=QUAD)
    b = AIMOperator(m, g, k, near_radius=6, rules=QUAD, bypass=False)
    assert a.local and a.all_near and not b.local
    L, K = _dense(m, k)
    x = random_vector(m.nrwg, 1)
    for op, M in (("L", L), ("K", K)):
        ref = M @ x
        for o in (a, b):
            assert np.linalg.norm(o.matvec(x, op) - ref) < 1e-12 * np.linalg.norm(ref), op


@pytest.fixture(scope="module")
def conductor():
    # conducting box (3 x 2 x 2 mm), sigma 1e5 S/m at 1 GHz: skin depth 50 um,
    # 5 skin depths well inside the near region (R h = 1 mm)
    m = RWGMesh([box_mesh((3e-3, 2e-3, 2e-3), (6, 4, 4))])
    k = ph.wavenumber(1e9, 1.0, 1.0, 1e5)
    g = Grid.enclosing(m.xyz, 12)
    return m, k, g


def test_skin_cutoff_within_decay_of_dense(conductor):
    m, k, g = conductor
    dc = 5.0 * ph.skin_depth(k)
    c = AIMOperator(m, g, k, near_radius=3, rules=QUAD, cutoff=dc)
    full = AIMOperator(m, g, k, near_radius=3, rules=QUAD)
    assert c.cut_local and not full.local
    # fewer pairs, and every dropped pair is farther apart than the cutoff
    assert len(c.near_t) < 0.6 * len(full.near_t)
    kept = set(zip(c.near_t.tolist(), c.near_s.tolist()))
    drop = np.array([i for i, p in enumerate(zip(full.near_t.tolist(), full.near_s.tolist())) if p not in kept])
    tl, sl = full.near_t[drop], full.near_s[drop]
    sep = np.linalg.norm(m.centroid[tl] - m.centroid[sl], axis=1) - c.rho[tl] - c.rho[sl]
    assert sep.min() > dc
    # the dropped interactions decay as exp(-sep / delta) / sep: 1e-7 of the product
    L, K = _dense(m, k)
    x = random_vector(m.nrwg, 2)
    for op, M in (("L", L), ("K", K)):
        ref = M @ x
        assert np.linalg.norm(c.matvec(x, op) - ref) < 1e-6 * np.linalg.norm(ref), op


def test_cutoff_beyond_near_region_keeps_the_grid(conductor):
    m, _, g = conductor
    k = ph.wavenumber(1e9, 1.0, 1.0, 10.0)        # skin depth 5 mm, beyond the 1 mm near region
    c = AIMOperator(m, g, k, near_radius=3, rules=QUAD, cutoff=5.0 * ph.skin_depth(k), near=False)
    assert not c.cut_local and not c.local
