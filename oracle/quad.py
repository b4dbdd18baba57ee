"""Triangle quadrature for the oracle: collapsed (Duffy) Gauss-Legendre rules.

An n x n rule maps the unit square to the triangle by x = u, y = v (1 - u);
it integrates polynomials of total degree <= 2n - 2 exactly.  The library
builds the same families of rules (collapsed Gauss-Legendre; corner, edge and
self rules for touching pairs) from its own code, with the same orders in the
parity tests: near-value parity between the two therefore checks that both
evaluate the same quadrature, while the correctness of that quadrature rests
on the closed-form, convergence and Mie pins of the oracle tests.
"""
import numpy as np


def collapsed_gauss(n):
    """Barycentric points [n*n, 3] and weights [n*n] summing to 1 (fractions of
    the triangle area) of the n x n collapsed Gauss-Legendre rule."""
    x, w = np.polynomial.legendre.leggauss(int(n))
    u = 0.5 * (x + 1.0)
    wu = 0.5 * w
    U, V = np.meshgrid(u, u, indexing="ij")
    WU, WV = np.meshgrid(wu, wu, indexing="ij")
    px = U.ravel()
    py = (V * (1.0 - U)).ravel()
    wt = (WU * WV * (1.0 - U)).ravel() * 2.0       # reference area 1/2 -> normalise to 1
    bary = np.stack([1.0 - px - py, px, py], axis=1)
    return bary, wt


def points_on(verts, bary):
    """Physical points: verts [...,3,3], bary [Q,3] -> [..., Q, 3]."""
    return np.einsum("qk,...kc->...qc", bary, verts)


def _gl01(n):
    x, w = np.polynomial.legendre.leggauss(int(n))
    return 0.5 * (x + 1.0), 0.5 * w


def corner_rule(n, V, Ev, F, q_rho=2, q_sig=3, frac=1.0):
    """Rule on the sub-triangle (V, Ev, F) given as barycentric 3-vectors of the
    parent triangle: collapsed at V (rho = u^q_rho) and graded towards the side
    V->Ev (sigma = v^q_sig), so that log singularities at V and along V->Ev
    become smooth in (u, v).  ``frac`` = sub-triangle area / parent area."""
    u, wu = _gl01(n)
    v, wv = _gl01(n)
    U, Vv = np.meshgrid(u, v, indexing="ij")
    WU, WV = np.meshgrid(wu, wv, indexing="ij")
    rho = (U ** q_rho).ravel()
    sig = (Vv ** q_sig).ravel()
    jac = (2.0 * rho * q_rho * U.ravel() ** (q_rho - 1) * q_sig * Vv.ravel() ** (q_sig - 1)
           * frac)
    V, Ev, F = (np.asarray(x, dtype=np.float64) for x in (V, Ev, F))
    bary = V[None, :] + rho[:, None] * ((1.0 - sig)[:, None] * (Ev - V)[None, :]
                                        + sig[:, None] * (F - V)[None, :])
    return bary, (WU * WV).ravel() * jac


def _e(i):
    e = np.zeros(3); e[i] = 1.0
    return e


def edge_graded(n, opp):
    """Rule for an edge-adjacent pair: the shared edge is opposite local vertex
    ``opp``; two sub-triangles (shared vertex, edge midpoint, opposite vertex),
    each collapsed at its shared vertex and graded towards the shared edge."""
    a, b = (opp + 1) % 3, (opp + 2) % 3
    m = 0.5 * (_e(a) + _e(b))
    r1 = corner_rule(n, _e(a), m, _e(opp), frac=0.5)
    r2 = corner_rule(n, _e(b), m, _e(opp), frac=0.5)
    return np.concatenate([r1[0], r2[0]]), np.concatenate([r1[1], r2[1]])


def vertex_collapsed(n, vtx, q=2):
    """Rule collapsed at local vertex ``vtx`` (radial coordinate rho = u^q),
    for vertex-adjacent pairs."""
    a, b = (vtx + 1) % 3, (vtx + 2) % 3
    return corner_rule(n, _e(vtx), _e(a), _e(b), q_rho=q, q_sig=1)


def self_fan(n):
    """Rule for the self pair: six sub-triangles (vertex, edge midpoint,
    centroid), each collapsed at its vertex and graded towards its edge."""
    g = np.full(3, 1.0 / 3.0)
    pts, wts = [], []
    for opp in range(3):
        a, b = (opp + 1) % 3, (opp + 2) % 3
        m = 0.5 * (_e(a) + _e(b))
        for v in (a, b):
            p, w = corner_rule(n, _e(v), m, g, frac=1.0 / 6.0)
            pts.append(p); wts.append(w)
    return np.concatenate(pts), np.concatenate(wts)
