"""Oracle pins for the AIM reference (Sec. III-D-1): direct-sum vs FFT
convolution, Lagrange moment identities, stencil geometry, agreement with the
dense operators, refinement, reciprocity, independence of the grid G(0)."""
import numpy as np
import pytest

from workloads import icosphere, box_mesh, random_vector
from oracle.rwg import RWGMesh
from oracle import mom
from oracle.aim import Grid, AIMOperator, stencil_centres, lagrange3, OFFS

K_TEST = 2.0 - 0.3j


@pytest.fixture(scope="module")
def sphere2():
    m = RWGMesh([icosphere(2)])
    A, P, K = mom.dense_operators(m, K_TEST)
    return m, {"A": A, "P": P, "K": K, "L": A - P / K_TEST ** 2}


def test_fft_convolution_equals_direct_sum():
    m = RWGMesh([icosphere(1)])
    op = AIMOperator(m, Grid.enclosing(m.xyz, 6), 3.0 - 1.0j, near_radius=2)
    x = random_vector(m.nrwg, 7)
    J, Q = op.project(x)
    for kind in ("G", 0, 1, 2):
        a = op.convolve_fft(Q, kind); b = op.convolve_direct(Q, kind)
        assert np.abs(a - b).max() < 1e-12 * np.abs(b).max()
    y1 = op.far_part(x, "K"); y2 = op.far_part(x, "K", conv=op.convolve_direct)
    assert np.abs(y1 - y2).max() < 1e-12 * np.abs(y2).max()


def test_lagrange_reproduces_quadratics():
    rng = np.random.default_rng(2)
    xi = rng.uniform(-0.5, 0.5, 50)
    l = lagrange3(xi)
    nodes = np.array([-1.0, 0.0, 1.0])
    for p in range(3):
        assert np.abs(l @ nodes ** p - xi ** p).max() < 1e-15


def test_moments_match_triangle_moments():
    """sum_a M0[t,a] = area; sum_a M0[t,a] x_a^p y_a^q z_a^r = int x^p y^q z^r dS
    for p, q, r <= 2 (moment matching, relative to the stencil centre)."""
    m = RWGMesh([icosphere(2)])
    g = Grid.enclosing(m.xyz, 10)
    op = AIMOperator(m, g, K_TEST, near_radius=1)
    from oracle.quad import collapsed_gauss, points_on
    b, w = collapsed_gauss(8)
    pts = points_on(m.verts, b) - g.node(op.centres)[:, None, :]
    offs = OFFS * g.h
    for p in range(3):
        for q in range(3):
            for r in range(3):
                lhs = op.M0 @ np.ones(27) if p + q + r == 0 else None
                lhs = np.einsum("ta,a->t", op.M0, offs[:, 0] ** p * offs[:, 1] ** q * offs[:, 2] ** r)
                rhs = np.einsum("q,tq,t->t", w, pts[..., 0] ** p * pts[..., 1] ** q * pts[..., 2] ** r, m.area)
                assert np.abs(lhs - rhs).max() < 1e-12 * max(np.abs(rhs).max(), m.area.max() * g.h ** (p + q + r))


def test_stencils_inside_and_centred():
    for xyz, tri in (icosphere(2), box_mesh((100e-6, 10e-6, 5e-6), (30, 3, 2))):
        m = RWGMesh([(xyz, tri)])
        g = Grid.enclosing(m.xyz, 16)
        c = stencil_centres(g, m.centroid)
        assert c.min() >= 1 and (c <= g.n - 2).all()
        off = np.abs(m.centroid - g.node(c)) / g.h
        assert off.max() <= 0.5 + 1e-12


@pytest.mark.parametrize("op_name", ["A", "P", "K", "L"])
def test_aim_matches_dense(sphere2, op_name):
    """AIM products within 3e-3 of the dense operators on a 12^3 grid with a
    7-point near region (kappa-type check, Sec. IV-A)."""
    m, dense = sphere2
    op = AIMOperator(m, Grid.enclosing(m.xyz, 12), K_TEST, near_radius=3)
    x = random_vector(m.nrwg, 11)
    y = op.matvec(x, op_name); yd = dense[op_name] @ x
    assert np.linalg.norm(y - yd) < 4e-3 * np.linalg.norm(yd)


def test_aim_error_falls_with_near_region(sphere2):
    m, dense = sphere2
    x = random_vector(m.nrwg, 12)
    errs = []
    for R in (2, 4):
        op = AIMOperator(m, Grid.enclosing(m.xyz, 12), K_TEST, near_radius=R)
        errs.append(np.linalg.norm(op.matvec(x, "L") - dense["L"] @ x))
    assert errs[1] < 0.5 * errs[0]


def test_aim_reciprocity():
    """x^T (A y) = y^T (A x) for the AIM operators (W = P^T, symmetric G)."""
    m = RWGMesh([icosphere(1)])
    op = AIMOperator(m, Grid.enclosing(m.xyz, 8), K_TEST, near_radius=2)
    x = random_vector(m.nrwg, 1); y = random_vector(m.nrwg, 2)
    for name, tol in (("A", 1e-6), ("P", 1e-6), ("K", 1e-4)):
        # grid part: exact structure (W = P^T, even G, odd grad G)
        a = x @ op.far_part(y, name); b = y @ op.far_part(x, name)
        assert abs(a - b) < 1e-12 * abs(a)
        # whole operator: up to the quadrature asymmetry of the direct near entries
        a = x @ op.matvec(y, name); b = y @ op.matvec(x, name)
        assert abs(a - b) < tol * abs(a)


def test_independent_of_grid_G0():
    m = RWGMesh([icosphere(1)])
    g = Grid.enclosing(m.xyz, 8)
    x = random_vector(m.nrwg, 3)
    y0 = AIMOperator(m, g, K_TEST, near_radius=2).matvec(x, "L")
    y1 = AIMOperator(m, g, K_TEST, near_radius=2, g0=123.0 - 45.0j).matvec(x, "L")
    assert np.abs(y0 - y1).max() < 1e-11 * np.abs(y0).max()


def test_direct_near_region_equals_dense_when_every_pair_is_near(sphere2):
    """The direct near-region L (source of the nested preconditioner,
    eq. nest2pc) is the dense L when the near region covers the object."""
    m, dense = sphere2
    op = AIMOperator(m, Grid.enclosing(m.xyz, 6), K_TEST, near_radius=10)
    N = op.NLd.toarray()
    assert np.abs(N - dense["L"]).max() < 1e-12 * np.abs(dense["L"]).max()


def test_direct_near_region_pattern_and_symmetry(sphere2):
    """Entries only where a triangle pair of the two RWG functions is near;
    symmetric up to quadrature (reciprocity); equal to the dense L on pairs
    whose every triangle pair is near."""
    m, dense = sphere2
    R = 2
    op = AIMOperator(m, Grid.enclosing(m.xyz, 12), K_TEST, near_radius=R)
    N = op.NLd.toarray()
    c = op.centres
    d = np.abs(c[:, None, :] - c[None, :, :]).max(axis=2)
    tp, tm = m.tp, m.tm
    any_near = np.zeros_like(N, bool); all_near = np.ones_like(N, bool)
    for a in (tp, tm):
        for b in (tp, tm):
            near = d[a][:, b] <= R
            any_near |= near; all_near &= near
    assert not np.any(N[~any_near])
    assert np.abs(N - N.T).max() < 1e-6 * np.abs(N).max()
    L = dense["L"]
    assert np.abs(N[all_near] - L[all_near]).max() < 1e-12 * np.abs(L).max()


def test_near_rows_equal_full_near_matrices():
    """Row-sampled near values (for meshes too large for the full matrices)
    reproduce the rows of the full near-region matrices."""
    m = RWGMesh([icosphere(2)])
    g = Grid.enclosing(m.xyz, 10)
    full = AIMOperator(m, g, K_TEST, near_radius=2)
    part = AIMOperator(m, g, K_TEST, near_radius=2, near=False)
    rows = np.random.default_rng(5).choice(m.nrwg, size=12, replace=False)
    got = part.near_rows(rows)
    L = full.near_L().tocsr(); K = full.NK.tocsr(); Ld = full.NLd.tocsr()
    for r in rows:
        cols, lv, kv, ldv = got[int(r)]
        for M, v in ((L, lv), (K, kv), (Ld, ldv)):
            row = M.getrow(r)
            row.sort_indices()
            nz = np.abs(row.toarray()[0]) > 0
            assert set(np.nonzero(nz)[0]) <= set(cols)
            assert np.abs(row.toarray()[0][cols] - v).max() <= 1e-14 * np.abs(M.data).max()
        assert np.array_equal(cols, np.sort(L.getrow(r).indices))
