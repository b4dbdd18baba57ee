"""AIM reference in FP64 (Sec. III-D-1, eq. AIM_Lin, AIM_Kin, LinNRP, KinNRP).

  L ~ (L_NR - L_P) + W G P - k^-2 W_phi G P_phi        (scalar term subtracted:
                                                        W_phi = -P_phi^T)
  K ~ (K_NR - K_P) + W G_grad P

Readings taken where the paper only cites the construction:

* Grid: isotropic spacing h = (largest bounding-box extent)/(N - 1 - 2m), margin
  m = 1, centred on the bounding box: x0 = centre - h (N - 1)/2.
* Stencil: order n = 2 (3 points per axis, 27 nodes), anchored per triangle at
  i = floor((c - x0)/h + 0.5) of the centroid c = ((v0 + v1) + v2)/3, clamped to
  [1, N - 2]; nodes i-1..i+1.
* Projection weights: Galerkin moments of the tensor Lagrange polynomials of the
  stencil, P_n(a) = int f_n l_a dS, P_phi,n(a) = int div f_n l_a dS, which match
  all monomial moments up to degree 2 per axis; interpolation W = P^T.
* Grid Green's function G[d] = G_k(h |d|) for d != 0 and 0 at d = 0; grad G
  likewise (the d = 0 value only touches overlapping stencils, which are near
  pairs and precorrected away).
* Near region: triangles t, s are near iff max_axis |i_t - i_s| <= R (R = 5:
  a diameter of 11 grid points); corrections are per triangle pair.
* Skin-depth cutoff (Sec. V: interactions farther apart than five skin depths
  are ignored), for a medium given the cutoff distance d_c: two triangles are
  "apart" when the distance of their centroids exceeds d_c + rho_t + rho_s,
  rho being a triangle's largest vertex distance from its centroid (so that
  touching triangles, whose minimum distance is zero, are never dropped).
  Applied where it removes the grid part: every far pair (centroids at least
  R h apart along some axis) is then beyond the cutoff, i.e. when
  d_c <= R h - 2 max(rho).  The operator is then the direct near-region one
  on the pairs within the cutoff (Sec. III-D-2 item a: L_NR = L once the skin
  depth is within the near region).
* Small objects (Sec. III-D-2 item b): when every pair of the grid is near
  (stencil centres within R of each other on every axis) the grid part equals
  the precorrection exactly, and the operator is the direct one.
"""
import numpy as np
import scipy.sparse as sp

from .quad import collapsed_gauss, points_on
from .mom import pair_blocks

FOUR_PI = 4.0 * np.pi


class Grid:
    def __init__(self, origin, h, n):
        self.origin = np.asarray(origin, dtype=np.float64)
        self.h = float(h)
        self.n = np.asarray(n, dtype=np.int64)

    @classmethod
    def enclosing(cls, xyz, n, margin=1):
        lo = xyz.min(axis=0); hi = xyz.max(axis=0)
        h = (hi - lo).max() / (n - 1 - 2 * margin)
        c = 0.5 * (lo + hi)
        return cls(c - h * (n - 1) / 2.0, h, (n, n, n))

    def node(self, idx):
        return self.origin + self.h * np.asarray(idx, dtype=np.float64)


def stencil_centres(grid, centroids):
    """Integer stencil centre per triangle (bit-exact with the library)."""
    q = (centroids - grid.origin) / grid.h
    i = np.floor(q + 0.5).astype(np.int64)
    return np.clip(i, 1, grid.n - 2)


def lagrange3(xi):
    """Lagrange polynomials on nodes -1, 0, 1 at local coordinate xi."""
    return np.stack([0.5 * xi * (xi - 1.0), 1.0 - xi * xi, 0.5 * xi * (xi + 1.0)], axis=-1)


OFFS = np.array([(a, b, c) for c in (-1, 0, 1) for b in (-1, 0, 1) for a in (-1, 0, 1)],
                dtype=np.int64)   # 27 stencil offsets, x fastest


def triangle_moments(mesh, grid, centres, nq=5):
    """M0[t, a] = int_t l_a dS and M1[t, a] = int_t l_a (r - r_centre) dS for
    the 27 nodes a of the stencil of t (x fastest)."""
    bary, w = collapsed_gauss(nq)                         # exact to degree 8
    pts = points_on(mesh.verts, bary)                     # [T,Q,3]
    rc = grid.node(centres)                               # [T,3]
    loc = (pts - rc[:, None, :]) / grid.h                 # [T,Q,3]
    lx = lagrange3(loc[..., 0]); ly = lagrange3(loc[..., 1]); lz = lagrange3(loc[..., 2])
    la = (lx[:, :, None, None, :] * ly[:, :, None, :, None] * lz[:, :, :, None, None])
    la = la.reshape(la.shape[0], la.shape[1], 27)         # [T,Q,27] index (c,b,a) -> x fastest
    W = w[None, :] * mesh.area[:, None]
    M0 = np.einsum("tq,tqa->ta", W, la)
    M1 = np.einsum("tq,tqa,tqc->tac", W, la, pts - rc[:, None, :])
    return M0, M1


def rwg_weights(mesh, grid, centres, M0, M1):
    """Per (triangle, local edge) projection weights:
    Pv[t, e, a, c] (vector) and Ps[t, e, a] (divergence)."""
    rc = grid.node(centres)
    sg = mesh.tri_sign * mesh.tri_len / (2.0 * mesh.area)[:, None]          # [T,3]
    pe = mesh.verts - rc[:, None, :]                                          # free vertex rel. centre
    Pv = sg[:, :, None, None] * (M1[:, None, :, :] - pe[:, :, None, :] * M0[:, None, :, None])
    Ps = (2.0 * sg)[:, :, None] * M0[:, None, :]
    return Pv, Ps


def node_index(grid, centres):
    """Global multi-index of the 27 nodes of every stencil [T,27,3]."""
    return centres[:, None, :] + OFFS[None, :, :]


def green_grid(k, h, d, g0=0.0):
    """G_k(h |d|) with the value g0 (default 0) at d = 0; d integer [...,3]."""
    r = h * np.linalg.norm(d, axis=-1)
    with np.errstate(divide="ignore", invalid="ignore"):
        g = np.exp(-1j * k * r) / (FOUR_PI * r)
    return np.where(r == 0, g0, g)


def grad_green_grid(k, h, d):
    """grad_r G_k at r = h d (observation minus source) with 0 at d = 0."""
    rv = h * np.asarray(d, dtype=np.float64)
    r = np.linalg.norm(rv, axis=-1)
    with np.errstate(divide="ignore", invalid="ignore"):
        s = -(1.0 + 1j * k * r) * np.exp(-1j * k * r) / (FOUR_PI * r ** 3)
    s = np.where(r == 0, 0.0, s)
    return s[..., None] * rv


class AIMOperator:
    """AIM approximations of A, Phi and K at one wavenumber on one grid."""

    def __init__(self, mesh, grid, k, near_radius=5, tris=None, rules=None, g0=0.0, near=True, cutoff=None,
                 bypass=True):
        self.mesh, self.grid, self.k, self.R = mesh, grid, complex(k), int(near_radius)
        self.g0 = g0                      # grid G at zero offset (result must not depend on it)
        T = len(mesh.tri)
        self.tris = np.arange(T) if tris is None else np.asarray(tris)
        self.centres = stencil_centres(grid, mesh.centroid)
        # local operator: no grid part (cutoff within the near region, or
        # every pair near)
        c = self.centres[self.tris]
        self.all_near = bypass and bool(np.all(c.max(axis=0) - c.min(axis=0) <= self.R))
        d = mesh.verts - mesh.centroid[:, None, :]
        self.rho = np.sqrt(np.max(np.sum(d * d, axis=2), axis=1))       # [T]
        self.cutoff = None if cutoff is None else float(cutoff)
        self.cut_local = self.cutoff is not None and \
            self.cutoff <= self.R * grid.h - 2.0 * float(self.rho[self.tris].max())
        self.local = self.all_near or self.cut_local
        self.M0, self.M1 = triangle_moments(mesh, grid, self.centres)
        self.Pv, self.Ps = rwg_weights(mesh, grid, self.centres, self.M0, self.M1)
        self.nodes = node_index(grid, self.centres)
        if np.any(self.nodes < 0) or np.any(self.nodes >= grid.n):
            raise ValueError("stencil outside grid")
        self.rules = rules
        if near:        # near=False: grid stages only (near rows on demand, near_rows)
            self.near_t, self.near_s = self.near_pairs()
            self._near_matrices(rules)

    # -- near region -------------------------------------------------------
    def near_pairs(self):
        c = self.centres[self.tris]
        d = np.abs(c[:, None, :] - c[None, :, :]).max(axis=2)
        ti, si = np.nonzero(d <= self.R)
        tl, sl = self.tris[ti], self.tris[si]
        if self.cut_local:
            keep = self.within_cutoff(tl, sl)
            tl, sl = tl[keep], sl[keep]
        return tl, sl

    def within_cutoff(self, tl, sl):
        """Pairs not farther apart than the cutoff (bounding spheres)."""
        dc = self.mesh.centroid[tl] - self.mesh.centroid[sl]
        lim = self.cutoff + self.rho[tl] + self.rho[sl]
        return np.sum(dc * dc, axis=1) <= lim * lim

    def near_rows(self, rows):
        """Precorrected near-region L and K (and direct L) of the given RWG rows
        only, for meshes too large for the full near matrices: for each row,
        its two triangles against every triangle of the grid within the near
        radius.  Returns {row: (cols ascending, L, K, L direct)}."""
        m = self.mesh
        k2 = self.k * self.k
        tset = np.unique(np.concatenate([m.tp[rows], m.tm[rows]]))
        c = self.centres
        tl, sl = [], []
        for t in tset:
            d = np.abs(c[self.tris] - c[t]).max(axis=1)
            ss = self.tris[d <= self.R]
            tl.append(np.full(len(ss), t)); sl.append(ss)
        tl = np.concatenate(tl); sl = np.concatenate(sl)
        if self.cut_local:
            keep = self.within_cutoff(tl, sl)
            tl, sl = tl[keep], sl[keep]
        Ad, Pd, Kd = pair_blocks(m, self.k, tl, sl, self.rules)
        Ag = np.zeros_like(Ad); Pg = np.zeros_like(Pd); Kg = np.zeros_like(Kd)
        if not self.local:
            for c0 in range(0, len(tl), 2000):
                Ag[c0:c0 + 2000], Pg[c0:c0 + 2000], Kg[c0:c0 + 2000] = self.grid_blocks(tl[c0:c0 + 2000],
                                                                                     sl[c0:c0 + 2000])
        Lp = (Ad - Ag) - (Pd - Pg) / k2
        Kp = Kd - Kg
        Ld = Ad - Pd / k2
        out = {}
        for r in rows:
            acc = {}
            for t, e in ((m.tp[r], m.ep[r]), (m.tm[r], m.em[r])):
                sel = np.nonzero(tl == t)[0]
                for pi in sel:
                    for f in range(3):
                        n = m.tri_rwg[sl[pi], f]
                        a = acc.setdefault(n, np.zeros(3, np.complex128))
                        a += (Lp[pi, e, f], Kp[pi, e, f], Ld[pi, e, f])
            cols = np.array(sorted(acc))
            vals = np.array([acc[n] for n in cols])
            out[int(r)] = (cols, vals[:, 0], vals[:, 1], vals[:, 2])
        return out

    def _offset_tables(self):
        """G and grad G on all node offsets a near pair can produce."""
        W = self.R + 2
        ax = np.arange(-W, W + 1)
        D = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), axis=-1)
        self._W = W
        self._Gt = green_grid(self.k, self.grid.h, D, self.g0)
        self._gGt = grad_green_grid(self.k, self.grid.h, D)

    def grid_blocks(self, tl, sl):
        """Grid contribution (P_t^T G P_s etc.) of triangle pairs: [P,3,3]."""
        if not hasattr(self, "_Gt"):
            self._offset_tables()
        dn = self.nodes[tl][:, :, None, :] - self.nodes[sl][:, None, :, :] + self._W   # [P,27,27,3]
        G = self._Gt[dn[..., 0], dn[..., 1], dn[..., 2]]
        gG = self._gGt[dn[..., 0], dn[..., 1], dn[..., 2]]                             # [P,27,27,3]
        Pt, Ps_ = self.Pv[tl], self.Pv[sl]                                    # [P,3,27,3]
        # A = sum_c Pt_c G Ps_c^T ; Phi = Pst G Pss^T
        A = sum(Pt[..., c] @ G @ np.swapaxes(Ps_[..., c], 1, 2) for c in range(3))
        Ph = self.Ps[tl] @ G @ np.swapaxes(self.Ps[sl], 1, 2)
        # K = sum_ab Pt(a) . (gradG(a-b) x Ps(b)) = sum_{c,i,j} eps_icj Pt_i gG_c Ps_j
        K = 0
        for c, i, j, s in ((0, 1, 2, -1), (0, 2, 1, 1), (1, 2, 0, -1), (1, 0, 2, 1),
                           (2, 0, 1, -1), (2, 1, 0, 1)):
            K = K + s * (Pt[..., i] @ gG[..., c] @ np.swapaxes(Ps_[..., j], 1, 2))
        return A, Ph, K

    def _near_matrices(self, rules, chunk=2000):
        E = self.mesh.nrwg
        rows, cols, va, vp, vk, vd = [], [], [], [], [], []
        self.direct_blocks = []
        for c0 in range(0, len(self.near_t), chunk):
            tl = self.near_t[c0:c0 + chunk]; sl = self.near_s[c0:c0 + chunk]
            Ad, Pd, Kd = pair_blocks(self.mesh, self.k, tl, sl, rules)
            if self.local:            # no grid part: nothing to precorrect
                Ag, Pg, Kg = np.zeros_like(Ad), np.zeros_like(Pd), np.zeros_like(Kd)
            else:
                Ag, Pg, Kg = self.grid_blocks(tl, sl)
            rm = self.mesh.tri_rwg[tl]; rn = self.mesh.tri_rwg[sl]
            rows.append(np.broadcast_to(rm[:, :, None], (len(tl), 3, 3)).ravel())
            cols.append(np.broadcast_to(rn[:, None, :], (len(tl), 3, 3)).ravel())
            va.append((Ad - Ag).ravel()); vp.append((Pd - Pg).ravel()); vk.append((Kd - Kg).ravel())
            vd.append((Ad - Pd / (self.k * self.k)).ravel())
        rows = np.concatenate(rows); cols = np.concatenate(cols)
        mk = lambda v: sp.coo_matrix((np.concatenate(v), (rows, cols)), shape=(E, E)).tocsr()
        self.NA, self.NP, self.NK = mk(va), mk(vp), mk(vk)
        # direct near-region L (no precorrection): L_NR of the paper's
        # near-region preconditioner (eq. nest2pc)
        self.NLd = mk(vd)
        for M in (self.NA, self.NP, self.NK, self.NLd):
            M.sum_duplicates()

    # -- grid stages ---------------------------------------------------------
    def project(self, x):
        """Grid sources: J [3, Nz, Ny, Nx] and Q [Nz, Ny, Nx] (x fastest)."""
        n = self.grid.n
        J = np.zeros((3, n[2], n[1], n[0]), np.complex128)
        Q = np.zeros((n[2], n[1], n[0]), np.complex128)
        xt = x[self.mesh.tri_rwg]                                             # [T,3]
        jv = np.einsum("te,teac->tac", xt, self.Pv)                           # [T,27,3]
        qs = np.einsum("te,tea->ta", xt, self.Ps)
        idx = self.nodes
        for c in range(3):
            np.add.at(J[c], (idx[..., 2], idx[..., 1], idx[..., 0]), jv[..., c])
        np.add.at(Q, (idx[..., 2], idx[..., 1], idx[..., 0]), qs)
        return J, Q

    def interpolate_vec(self, F):
        """y_m = sum_a P_m(a) . F(a) for a vector field F [3, Nz, Ny, Nx]."""
        idx = self.nodes
        f = np.stack([F[c][idx[..., 2], idx[..., 1], idx[..., 0]] for c in range(3)], axis=-1)
        yt = np.einsum("teac,tac->te", self.Pv, f)
        y = np.zeros(self.mesh.nrwg, np.complex128)
        np.add.at(y, self.mesh.tri_rwg, yt)
        return y

    def interpolate_scal(self, F):
        idx = self.nodes
        f = F[idx[..., 2], idx[..., 1], idx[..., 0]]
        yt = np.einsum("tea,ta->te", self.Ps, f)
        y = np.zeros(self.mesh.nrwg, np.complex128)
        np.add.at(y, self.mesh.tri_rwg, yt)
        return y

    def kernel_fft(self, kind):
        """Circulant embedding (2N per axis) of G or dG/dx_c on the offsets
        -(N-1)..(N-1), transformed: [2Nz, 2Ny, 2Nx] (kept per kind)."""
        cache = self.__dict__.setdefault("_kfft", {})
        if kind not in cache:
            cache[kind] = self._kernel_fft(kind)
        return cache[kind]

    def _kernel_fft(self, kind):
        n = self.grid.n
        m = 2 * n
        ax = [np.concatenate([np.arange(0, n[i]), [0], np.arange(-(n[i] - 1), 0)]) for i in range(3)]
        valid = [np.concatenate([np.ones(n[i], bool), [False], np.ones(n[i] - 1, bool)]) for i in range(3)]
        D = np.stack(np.meshgrid(ax[0], ax[1], ax[2], indexing="ij"), axis=-1)   # [mx,my,mz,3]
        V = valid[0][:, None, None] & valid[1][None, :, None] & valid[2][None, None, :]
        if kind == "G":
            g = green_grid(self.k, self.grid.h, D, self.g0)
        else:
            g = grad_green_grid(self.k, self.grid.h, D)[..., kind]
        g = np.where(V, g, 0.0)
        return np.fft.fftn(np.transpose(g, (2, 1, 0)))

    def convolve_fft(self, src, kind):
        n = self.grid.n
        m = 2 * n
        pad = np.zeros((m[2], m[1], m[0]), np.complex128)
        pad[:n[2], :n[1], :n[0]] = src
        out = np.fft.ifftn(np.fft.fftn(pad) * self.kernel_fft(kind))
        return out[:n[2], :n[1], :n[0]]

    def convolve_direct(self, src, kind):
        """O(N^6) direct sum (tiny grids only)."""
        n = self.grid.n
        zz, yy, xx = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
        pts = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)
        D = pts[:, None, :] - pts[None, :, :]
        if kind == "G":
            g = green_grid(self.k, self.grid.h, D, self.g0)
        else:
            g = grad_green_grid(self.k, self.grid.h, D)[..., kind]
        return (g @ src.ravel()).reshape(src.shape)

    def far_part(self, x, op, conv=None):
        if self.local:
            return np.zeros(self.mesh.nrwg, np.complex128)
        conv = conv or self.convolve_fft
        J, Q = self.project(x)
        if op == "A":
            return self.interpolate_vec(np.stack([conv(J[c], "G") for c in range(3)]))
        if op == "P":
            return self.interpolate_scal(conv(Q, "G"))
        if op == "K":
            d = [[conv(J[c], a) for c in range(3)] for a in range(3)]   # d[a][c] = dG/dx_a * J_c
            psi = np.stack([d[1][2] - d[2][1], d[2][0] - d[0][2], d[0][1] - d[1][0]])
            return self.interpolate_vec(psi)
        raise ValueError(op)

    def matvec(self, x, op, conv=None):
        """AIM product for op in A, P (Phi), K, L (= A - k^-2 Phi)."""
        if op == "L":
            return self.matvec(x, "A", conv) - self.matvec(x, "P", conv) / self.k ** 2
        near = {"A": self.NA, "P": self.NP, "K": self.NK}[op]
        return near @ x + self.far_part(x, op, conv)

    def near_L(self):
        return self.NA - self.NP / self.k ** 2
