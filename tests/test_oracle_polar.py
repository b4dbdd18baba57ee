"""Pins of the oracle's strong-loss inner integration (polar coordinates
around the projected observation point; oracle/csrc/pairint.c polar_pot):
independent brute force by subdivision of the source triangle, the closed
forms of the plane limit, agreement with the static-extraction scheme where
both are accurate, and the Mie series of a highly conducting sphere."""
import numpy as np
import pytest

from oracle._clib import polar_pot_c
from oracle.mom import inner_integrals, pair_blocks, polar_pairs, classify_pairs, KIND_CLOSE
from oracle.rwg import RWGMesh
from workloads import icosphere

TRI = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.3, 0.9, 0.0]])


def _subdivide(v, L):
    tris = [np.asarray(v, float)]
    for _ in range(L):
        nt = []
        for t in tris:
            a, b, c = t
            ab, bc, ca = (a + b) / 2, (b + c) / 2, (c + a) / 2
            nt += [np.array([a, ab, ca]), np.array([ab, b, bc]), np.array([ca, bc, c]), np.array([ab, bc, ca])]
        tris = nt
    return np.array(tris)


def _brute(v, r, k, L, n_in):
    """Sum of the static-extraction scheme over 4^L sub-triangles, each small
    enough (|k| l ~ 1) for that scheme."""
    sv = _subdivide(v, L)
    obs = np.broadcast_to(np.asarray(r, float), (len(sv), 1, 3)).copy()
    S, V, Gv = inner_integrals(k, sv, obs, n_in)
    return S.sum(), V.sum(axis=0)[0], Gv.sum(axis=0)[0]


@pytest.mark.parametrize("K", [20.0, 60.0])
@pytest.mark.parametrize("r", [[0.5, 0.004, 0.0], [0.4, 0.3, 0.03], [0.5, 0.01, -0.02],
                               [0.5, -0.02, 0.0], [0.4, 0.3, 0.4],
                               # off the plane, projected onto an edge (faces at right angles)
                               [0.5, 0.0, 0.03], [0.7, 0.0, -0.004]])
def test_polar_matches_subdivision(K, r):
    k = K * (1 - 1j) / np.sqrt(2)
    S, V, G = polar_pot_c(TRI, r, k)
    near_edge = abs(r[1]) < 0.011 and abs(r[2]) < 0.011
    # points within 0.01 of an edge are near-singular for the sub-triangles
    # too: finer subdivision there
    Sb, Vb, Gb = _brute(TRI, r, k, 7 if near_edge else 5, 12 if near_edge else 8)
    assert abs(S - Sb) < 2e-6 * max(abs(Sb), 1.0 / K)
    assert np.abs(V - Vb).max() < 2e-6 * max(np.abs(Vb).max(), 1.0 / K)
    assert np.abs(G - Gb).max() < (2e-5 if near_edge else 1e-5)


@pytest.mark.parametrize("K", [20.0, 60.0])
def test_polar_in_plane_interior_point(K):
    """The kink of the remainder at an in-plane point needs a fine brute force."""
    k = K * (1 - 1j) / np.sqrt(2)
    r = [0.4, 0.3, 0.0]
    S, V, G = polar_pot_c(TRI, r, k)
    Sb, Vb, Gb = _brute(TRI, r, k, 7, 8)
    assert abs(S - Sb) < 2e-6 * abs(Sb)
    assert np.abs(V - Vb).max() < 2e-6 * np.abs(Vb).max()
    assert np.abs(G - Gb).max() < 5e-5


@pytest.mark.parametrize("d", [0.0, 2e-4, -5e-4])
def test_polar_plane_limit(d):
    """|k| l = 1e4: far from the edges the triangle is a plane; int G over a
    plane at height d is exp(-jk|d|)/(2jk), int grad G . n is
    -sign(d) exp(-jk|d|)/2, the tangential gradient vanishes and V = rho0 S."""
    k = 1e4 * (1 - 1j) / np.sqrt(2)
    r = np.array([0.4, 0.3, d])
    S, V, G = polar_pot_c(TRI, r, k)
    e = np.exp(-1j * k * abs(d))
    assert abs(S - e / (2j * k)) < 1e-9 * abs(1 / (2 * k))
    assert np.abs(V - np.array([0.4, 0.3, 0.0]) * S).max() < 1e-9 * abs(S)
    assert abs(G[2] - (-np.sign(d) * e / 2)) < 1e-9
    assert np.abs(G[:2]).max() < 1e-9


def test_polar_blocks_match_extraction_where_both_hold():
    """|Im k| l = 3: the polar scheme and the static-extraction scheme with
    16x16 inner rules give the same Galerkin blocks to the extraction's own
    convergence level (~1e-4; scale: the largest block of each operator,
    coplanar self blocks of K being zero up to rounding)."""
    from oracle._clib import pair_blocks_c
    from oracle.mom import outer_rule, inner_rule, DEFAULT_RULES
    m = RWGMesh([icosphere(1)])
    k = (3.0 / m.tri_len.max()) * (1 - 1j)
    T = len(m.tri)
    tl = np.repeat(np.arange(T), T); sl = np.tile(np.arange(T), T)
    kind, local = classify_pairs(m, tl, sl)
    sel = polar_pairs(m, k, sl, kind) & (kind <= KIND_CLOSE)
    assert sel.sum() > 0
    tl, sl, kind, local = tl[sel], sl[sel], kind[sel], local[sel]
    got = pair_blocks(m, k, tl, sl)
    ref = [np.empty_like(got[0]) for _ in range(3)]
    hi = dict(DEFAULT_RULES, touch_in=16, close_in=16)
    for kd in range(4):
        for lc in ((0,) if kd in (0, 3) else range(3)):
            idx = np.nonzero((kind == kd) & ((local == lc) | (kd in (0, 3))))[0]
            if len(idx):
                out = pair_blocks_c(m, k, tl[idx], sl[idx], outer_rule(kd, lc, hi), inner_rule(kd, hi))
                for j in range(3):
                    ref[j][idx] = out[j]
    for X, Y in zip(got, ref):
        assert np.abs(X - Y).max() < 2e-4 * np.abs(Y).max()


def test_polar_scheme_selection():
    m = RWGMesh([icosphere(1)])
    T = len(m.tri)
    tl = np.repeat(np.arange(T), T); sl = np.tile(np.arange(T), T)
    kind, _ = classify_pairs(m, tl, sl)
    lmax = m.tri_len.max()
    assert not polar_pairs(m, 100.0 / lmax, sl, kind).any()            # lossless
    assert not polar_pairs(m, (1.0 / lmax) * (1 - 1j), sl, kind).any()  # mildly lossy
    assert polar_pairs(m, (50.0 / lmax) * (1 - 1j), sl, kind).all()


@pytest.mark.parametrize("level,sigma,tol", [(2, 100.0, 0.08), (2, 1e4, 0.08)])
def test_absorbed_power_of_conducting_sphere_matches_mie(level, sigma, tol):
    """Power entering a highly conducting sphere (skin depth 1e-2 to 1e-3 of
    the mesh edge), 1/2 Re(u^H X v) from the surface currents, against the
    Mie absorption cross-section: first order in the surface impedance, so it
    checks the interior operator itself (the scattered field alone tends to
    the PEC limit whatever the interior operator is).  At 320 triangles the
    ratio is 0.94 for both conductivities (1,280 triangles: 0.985); the static
    extraction gave 0.64 and -0.24."""
    from oracle import physics as ph, mie
    from oracle.solve import DenseProblem
    F = 150e6
    m = RWGMesh([icosphere(level)])
    dp = DenseProblem(m, F, [(4.0, 1.0, sigma)])
    u, v = dp.solve_block(dp.rhs((0.0, 0.0, 1.0), (1.0, 0.0, 0.0)))
    p_in = 0.5 * np.real(np.conj(u) @ (dp.X @ v))
    ce, cs = mie.cross_sections(dp.k0, 1.0, ph.eps_tilde(F, 4.0, sigma) / ph.EPS0)
    p_mie = (ce - cs) / (2 * dp.eta0)
    assert abs(p_in / p_mie - 1.0) < tol
