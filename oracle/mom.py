"""Dense Galerkin method of moments for the operators of Sec. III-A/B.

Operators (eq. opL, eq. opK, eq. Grrpki), tested with RWG functions:

  L^k_mn = A_mn - k^-2 Phi_mn
  A_mn   = int int f_m . f_n  G dS' dS
  Phi_mn = int int (div f_m)(div' f_n) G dS' dS
  K^k_mn = int f_m . PV int grad_r G(r - r') x f_n(r') dS' dS
  X_mn   = int (n x f_m) . f_n dS             (the identity operator the paper
                                               writes as I-cross, tested with RWG)
  e_m    = int f_m . E_inc dS

with G = exp(-j k R)/(4 pi R).  The paper's grad'grad'. in eq. opL is read as
k^-2 grad (div' X), which after integration by parts on the closed surface gives
the -k^-2 Phi term.  The Galerkin K needs no principal-value care: the
observation points are interior quadrature points and the 1/2 jump terms are
carried separately by X.

Integration: for every triangle pair the inner integral over the source
triangle splits G = 1/(4 pi R) + [G - 1/(4 pi R)]; the first part is integrated
in closed form (``static``), the bounded remainder with a collapsed Gauss rule.
"""
import numpy as np

from .quad import collapsed_gauss, points_on, self_fan, edge_graded, vertex_collapsed
from .static import triangle_potentials

FOUR_PI = 4.0 * np.pi


def expm1_c(z):
    """exp(z) - 1 for complex z without cancellation."""
    a, b = z.real, z.imag
    return np.expm1(a) * np.cos(b) - 2.0 * np.sin(0.5 * b) ** 2 + 1j * np.exp(a) * np.sin(b)


def one_minus_1pz_exp(z):
    """1 - (1 - z) exp(z) for complex z (z = -j k R): sum_{n>=2} (n-1) z^n / n!
    for |z| < 1, direct otherwise."""
    z = np.asarray(z, dtype=np.complex128)
    out = np.empty_like(z)
    small = np.abs(z) < 1.0
    zs = z[small]
    acc = np.zeros_like(zs)
    term = zs * zs / 2.0               # z^n / n! at n = 2
    for n in range(2, 30):
        acc += (n - 1) * term
        term = term * zs / (n + 1)
    out[small] = acc
    zl = z[~small]
    out[~small] = -expm1_c(zl) + zl * np.exp(zl)
    return out


def inner_integrals(k, sverts, obs, n_in):
    """For source triangles sverts [P,3,3] and observation points obs [P,Q,3]:

      S  = int_s G dS'                       [P,Q]
      V  = int_s G r' dS'                    [P,Q,3]
      Gv = int_s grad_r G(r - r') dS'        [P,Q,3]
    """
    I, Irho, gI = triangle_potentials(sverts, obs)
    v0, v1, v2 = sverts[:, 0], sverts[:, 1], sverts[:, 2]
    n = np.cross(v1 - v0, v2 - v0)
    A = 0.5 * np.linalg.norm(n, axis=1)
    n = n / (2.0 * A)[:, None]
    d = np.einsum("pqc,pc->pq", obs - v0[:, None, :], n)
    d = np.where(np.abs(d) <= 1e-10 * np.linalg.norm(v1 - v0, axis=1)[:, None], 0.0, d)
    rho = obs - d[..., None] * n[:, None, :]
    S = I / FOUR_PI
    V = (Irho + rho * I[..., None]) / FOUR_PI
    Gv = gI / FOUR_PI
    bary, w = collapsed_gauss(n_in)
    P = points_on(sverts, bary)                          # [P,Qi,3]
    diff = obs[:, :, None, :] - P[:, None, :, :]         # r - r'  [P,Q,Qi,3]
    R = np.linalg.norm(diff, axis=3)
    z = -1j * k * R
    wA = (w[None, :] * A[:, None])[:, None, :]          # [P,1,Qi]
    zero = R == 0.0
    Rs = np.where(zero, 1.0, R)
    # G - 1/(4 pi R), whose limit at R = 0 is -j k/(4 pi)
    rem = np.where(zero, -1j * k / FOUR_PI, expm1_c(z) / (FOUR_PI * Rs))
    S = S + np.sum(wA * rem, axis=2)
    V = V + np.einsum("pqi,pic->pqc", wA * rem, P)
    # grad G - grad 1/(4 pi R) = (r - r') hg; the product vanishes at R = 0
    hg = np.where(zero, 0.0, one_minus_1pz_exp(z) / (FOUR_PI * Rs ** 3))
    Gv = Gv + np.einsum("pqi,pqic->pqc", wA * hg, diff)
    return S, V, Gv


def pair_blocks_np(mesh, k, tl, sl, n_out=5, n_in=5):
    """Local 3x3 blocks (test edge e of t, source edge f of s) of A, Phi and K
    for the triangle pairs (tl[p], sl[p]); numpy version, used to cross-check
    the C version on small cases."""
    tl = np.asarray(tl); sl = np.asarray(sl)
    tv = mesh.verts[tl]; sv = mesh.verts[sl]
    bary, w = collapsed_gauss(n_out)
    obs = points_on(tv, bary)                            # [P,Qo,3]
    S, V, Gv = inner_integrals(k, sv, obs, n_in)
    W = w[None, :] * mesh.area[tl][:, None]              # [P,Qo]
    ct = mesh.tri_sign[tl] * mesh.tri_len[tl] / (2.0 * mesh.area[tl])[:, None]   # [P,3]
    cs = mesh.tri_sign[sl] * mesh.tri_len[sl] / (2.0 * mesh.area[sl])[:, None]
    dt = 2.0 * ct
    ds = 2.0 * cs
    rt = obs[:, :, None, :] - tv[:, None, :, :]          # r_q - p_t[e]  [P,Qo,3,3]
    ps = sv                                              # p_s[f] [P,3,3]
    # int_s G (r' - p_f) = V - p_f S
    Vf = V[:, :, None, :] - ps[:, None, :, :] * S[..., None, None]     # [P,Qo,3f,3]
    Aloc = np.einsum("pq,pqec,pqfc->pef", W, rt, Vf) * ct[:, :, None] * cs[:, None, :]
    Ploc = np.einsum("pq,pq->p", W, S)[:, None, None] * dt[:, :, None] * ds[:, None, :]
    rs = obs[:, :, None, :] - ps[:, None, :, :]          # r_q - p_s[f]
    cr = np.cross(Gv[:, :, None, :], rs)                 # Gv x (r - p_f)  [P,Qo,3f,3]
    Kloc = np.einsum("pq,pqec,pqfc->pef", W, rt, cr) * ct[:, :, None] * cs[:, None, :]
    return Aloc, Ploc, Kloc


# Integration policy of the oracle.  Pairs are classified by their relation:
# self, edge-adjacent, vertex-adjacent, close (centroid distance below
# CLOSE_FACTOR times the longest edge of either), far.  Touching pairs use outer
# rules adapted to the shared feature (``quad.self_fan``, ``quad.edge_graded``,
# ``quad.vertex_collapsed``); the others collapsed Gauss rules.
DEFAULT_RULES = dict(touch_out=10, touch_in=8, close_out=8, close_in=8, far_out=5, far_in=5)
CLOSE_FACTOR = 2.5
KIND_SELF, KIND_EDGE, KIND_VERTEX, KIND_CLOSE, KIND_FAR = range(5)


def classify_pairs(mesh, tl, sl):
    """Returns (kind [P], local [P]) where local is the local vertex of t that
    is opposite the shared edge (edge-adjacent) or the shared vertex of t
    (vertex-adjacent)."""
    tl = np.asarray(tl); sl = np.asarray(sl)
    match = np.zeros((len(tl), 3), bool)                 # vertex i of t is shared
    for a in range(3):
        for b in range(3):
            match[:, a] |= mesh.tri[tl, a] == mesh.tri[sl, b]
    ns = match.sum(1)
    d = np.linalg.norm(mesh.centroid[tl] - mesh.centroid[sl], axis=1)
    hmax = np.maximum(mesh.tri_len[tl].max(1), mesh.tri_len[sl].max(1))
    kind = np.full(len(tl), KIND_FAR)
    kind[d < CLOSE_FACTOR * hmax] = KIND_CLOSE
    kind[ns == 1] = KIND_VERTEX
    kind[ns == 2] = KIND_EDGE
    kind[ns == 3] = KIND_SELF
    local = np.zeros(len(tl), np.int64)
    local[ns == 1] = np.argmax(match[ns == 1], axis=1)
    local[ns == 2] = np.argmin(match[ns == 2], axis=1)
    return kind, local


def outer_rule(kind, local, rules):
    n = rules["touch_out"]
    if kind == KIND_SELF:
        return self_fan(n)
    if kind == KIND_EDGE:
        return edge_graded(n, local)
    if kind == KIND_VERTEX:
        return vertex_collapsed(n, local)
    if kind == KIND_CLOSE:
        return collapsed_gauss(rules["close_out"])
    return collapsed_gauss(rules["far_out"])


def inner_rule(kind, rules):
    if kind in (KIND_SELF, KIND_EDGE, KIND_VERTEX):
        return collapsed_gauss(rules["touch_in"])
    if kind == KIND_CLOSE:
        return collapsed_gauss(rules["close_in"])
    return collapsed_gauss(rules["far_in"])


# Strong loss: G decays within a fraction of a triangle and the static
# extraction cancels to far below its parts (for distant pairs the true value
# is exponentially small and the extraction leaves its quadrature error).
# Pairs whose source triangle's longest edge l has |Im k| l > POLAR_KL, in
# media with |Im k| >= POLAR_LOSS |k|, take the polar inner scheme
# (oracle/csrc/pairint.c), whatever their kind.
POLAR_KL = 2.0
POLAR_LOSS = 0.38


def polar_pairs(mesh, k, sl, kind=None):
    """Boolean [P]: pairs integrated with the strong-loss inner scheme."""
    k = complex(k)
    if abs(k.imag) < POLAR_LOSS * abs(k):
        return np.zeros(len(sl), bool)
    lmax = mesh.tri_len[np.asarray(sl)].max(axis=1)
    return abs(k.imag) * lmax > POLAR_KL


def pair_blocks(mesh, k, tl, sl, rules=None):
    """Local (A, Phi, K) blocks [P,3,3] with the oracle's integration policy
    (plain-C core)."""
    from ._clib import pair_blocks_c
    r = dict(DEFAULT_RULES)
    if rules:
        r.update(rules)
    tl = np.asarray(tl, dtype=np.int64); sl = np.asarray(sl, dtype=np.int64)
    kind, local = classify_pairs(mesh, tl, sl)
    pol = polar_pairs(mesh, k, sl, kind)
    P = len(tl)
    A = np.empty((P, 3, 3), np.complex128); Ph = np.empty_like(A); K = np.empty_like(A)
    for kd in range(5):
        for lc in (range(3) if kd in (KIND_EDGE, KIND_VERTEX) else (0,)):
            sel = (kind == kd) if kd not in (KIND_EDGE, KIND_VERTEX) else ((kind == kd) & (local == lc))
            for pl in (False, True):
                idx = np.nonzero(sel & (pol == pl))[0]
                if len(idx) == 0:
                    continue
                a, p, kk = pair_blocks_c(mesh, k, tl[idx], sl[idx], outer_rule(kd, lc, r),
                                         inner_rule(kd, r), polar=pl)
                A[idx] = a; Ph[idx] = p; K[idx] = kk
    return A, Ph, K


def scatter_blocks(mesh, M, tl, sl, blk):
    """M[m, n] += blk[p, e, f] for m = rwg(tl[p], e), n = rwg(sl[p], f)."""
    rm = mesh.tri_rwg[tl]                                # [P,3]
    rn = mesh.tri_rwg[sl]
    np.add.at(M, (rm[:, :, None], rn[:, None, :]), blk)


def dense_operators(mesh, k, obj=None, rules=None, chunk_pairs=2_000_000):
    """Dense A, Phi, K (complex [E,E]) at wavenumber k.  With ``obj`` given, only
    triangle pairs inside that object contribute (interior medium of the
    object); otherwise all pairs (exterior medium)."""
    E = mesh.nrwg
    A = np.zeros((E, E), np.complex128)
    P = np.zeros((E, E), np.complex128)
    K = np.zeros((E, E), np.complex128)
    T = len(mesh.tri)
    tris = np.arange(T) if obj is None else np.nonzero(mesh.tri_obj == obj)[0]
    nt = len(tris)
    rows = max(1, chunk_pairs // nt)
    for c0 in range(0, nt, rows):
        tt = tris[c0:c0 + rows]
        tl = np.repeat(tt, nt); sl = np.tile(tris, len(tt))
        a, p, kk = pair_blocks(mesh, k, tl, sl, rules)
        scatter_blocks(mesh, A, tl, sl, a)
        scatter_blocks(mesh, P, tl, sl, p)
        scatter_blocks(mesh, K, tl, sl, kk)
    return A, P, K


def L_from(A, P, k):
    """L^k = A - k^-2 Phi."""
    return A - P / (k * k)


def x_matrix(mesh):
    """X_mn = int (n x f_m) . f_n dS (sparse in nature, returned dense)."""
    E = mesh.nrwg
    X = np.zeros((E, E))
    bary, w = collapsed_gauss(3)
    T = len(mesh.tri)
    tl = np.arange(T)
    pts = points_on(mesh.verts, bary)                    # [T,Q,3]
    c = mesh.tri_sign * mesh.tri_len / (2.0 * mesh.area)[:, None]
    f = c[:, None, :, None] * (pts[:, :, None, :] - mesh.verts[:, None, :, :])  # [T,Q,3,3]
    nf = np.cross(mesh.normal[:, None, None, :], f)
    loc = np.einsum("q,tqec,tqfc->tef", w, nf, f) * mesh.area[:, None, None]
    scatter_blocks(mesh, X, tl, tl, loc)
    return X


def excitation(mesh, k0, khat, e0, n_q=6):
    """e_m = int f_m . E_inc dS with E_inc = e0 exp(-j k0 khat . r)."""
    bary, w = collapsed_gauss(n_q)
    pts = points_on(mesh.verts, bary)                    # [T,Q,3]
    ph = np.exp(-1j * k0 * np.einsum("tqc,c->tq", pts, np.asarray(khat, float)))
    einc = ph[..., None] * np.asarray(e0, dtype=np.complex128)[None, None, :]
    c = mesh.tri_sign * mesh.tri_len / (2.0 * mesh.area)[:, None]
    f = c[:, None, :, None] * (pts[:, :, None, :] - mesh.verts[:, None, :, :])
    loc = np.einsum("q,tqec,tqc->te", w, f, einc) * mesh.area[:, None]
    out = np.zeros(mesh.nrwg, np.complex128)
    np.add.at(out, mesh.tri_rwg, loc)
    return out


def incident_h_projection(mesh, k0, eta0, khat, e0, n_q=6):
    """h_m = int f_m . H_inc dS with H_inc = (khat x E_inc)/eta0 (null-field test)."""
    h0 = np.cross(np.asarray(khat, float), np.asarray(e0, dtype=np.complex128)) / eta0
    return excitation(mesh, k0, khat, h0, n_q)
