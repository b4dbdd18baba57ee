"""Augmented EFIE of the exterior problem with the constraint preconditioner
(Sec. III-E, eq. sys).

Test infrastructure: see the package docstring for who may import it.

At low frequency the scalar potential of the exterior L0 outweighs its vector
potential by about (k0 h)^-2, and the GIBC system (eq. GIBCsys) stalls in
plateaus.  The paper therefore takes the surface charge density as a further
unknown, expanded in pulses (one per triangle), and scales the exterior row by
1/eta0.  It leaves the sparse matrices D, B and F of eq. sys to the literature;
the reading used here, written with the divergence matrix

    Dv[t, n] = div f_n on triangle t   (+l_n/A_t on T+, -l_n/A_t on T-, 0 else;
                                        the product F D of the signed, length
                                        weighted incidence D and F = diag(1/A))

and the pulse-pulse potential integrals Gam[t, s] = int_t int_s G0 dS' dS, is

    Phi0 = Dv^T Gam Dv                      (scalar part of L0, eq. opL)
    sigma = c0 rho,  div J = -j w rho  =>   Dv u + j k0 sigma = 0

    [ j k0 A0 - (K0 - X/2) Z / eta0 ,  -Dv^T Gam ] [ u     ]   [ e / eta0 ]
    [ Dv                            ,   j k0 I   ] [ sigma ] = [ 0        ]

(w mu0 / eta0 = k0 and 1/(eps0 eta0) = c0 turn j w mu0 L0 u into j k0 A0 u -
Dv^T Gam sigma).  Eliminating sigma = -Dv u / (j k0) gives back the GIBC system
divided by eta0, so both have the same u (pinned in the tests).

Row weighting (a reading: the paper gives none).  The continuity row is
multiplied by A_t / k0.  Its terms then scale like those of the exterior row,
and the weighted residual measures what an error in the continuity row does to
the EFIE.  Without the weight that row dominates the residual norm by about
(k0 h)^-2 / h^2, and GMRES would stop before the exterior row converged.

The constraint preconditioner keeps j k0 diag(A0) in the (1,1) block (the
paper's choice) and, in this reading, the constraint blocks with the self
integrals of the triangles:

    P = [ j k0 diag(A0) , -Dv^T diag(Gam) ]
        [ Dv            ,  j k0 I         ]

Its Schur complement S = j k0 I + Dv diag(j k0 A0)^-1 Dv^T diag(Gam) has the
sparsity of the triangle adjacency and is solved exactly.
"""
import numpy as np

from .mom import pair_blocks
from .solve import DenseProblem


def divergence_matrix(mesh):
    """Dv [T, E]: surface divergence of RWG function n on triangle t (Sec. III-A
    RWG definition)."""
    T = len(mesh.tri)
    Dv = np.zeros((T, mesh.nrwg))
    for t in range(T):
        for e in range(3):
            n = mesh.tri_rwg[t, e]
            Dv[t, n] += mesh.tri_sign[t, e] * mesh.tri_len[t, e] / mesh.area[t]
    return Dv


def pulse_potentials(mesh, k, rules=None, chunk_pairs=2_000_000):
    """Gam [T, T] = int_t int_s G dS' dS at wavenumber k.  The oracle's pair
    integrals give the Phi block of a triangle pair as div f_e div f_f times
    this integral (eq. opL), so it is that block's (0, 0) entry divided by
    the two divergences."""
    T = len(mesh.tri)
    Gam = np.zeros((T, T), np.complex128)
    div0 = mesh.tri_sign[:, 0] * mesh.tri_len[:, 0] / mesh.area
    tris = np.arange(T)
    rows = max(1, chunk_pairs // T)
    for c0 in range(0, T, rows):
        tt = tris[c0:c0 + rows]
        tl = np.repeat(tt, T)
        sl = np.tile(tris, len(tt))
        _, ph, _ = pair_blocks(mesh, k, tl, sl, rules)
        Gam[tl, sl] = ph[:, 0, 0] / (div0[tl] * div0[sl])
    return Gam


def equilibrated_solve(M, b):
    """Dense solve of M x = b after scaling the rows, then the columns, of M to
    unit largest magnitude (keeps partial pivoting meaningful when the blocks
    of M differ in scale by many orders)."""
    r = 1.0 / np.abs(M).max(axis=1)
    Ms = M * r[:, None]
    c = 1.0 / np.abs(Ms).max(axis=0)
    return np.linalg.solve(Ms * c[None, :], b * r) * c


class AugmentedProblem(DenseProblem):
    """Dense blocks of eq. sys for a problem of DenseProblem (exterior at k0,
    interiors per object)."""

    def __init__(self, mesh, freq, materials, bg_eps_r=1.0, bg_mu_r=1.0, rules=None):
        super().__init__(mesh, freq, materials, bg_eps_r, bg_mu_r, rules)
        self.Dv = divergence_matrix(mesh)
        self.Gam0 = pulse_potentials(mesh, self.k0, rules)
        self.T = len(mesh.tri)

    @property
    def row_weight(self):
        """Weight A_t / k0 of the continuity rows (module docstring)."""
        return self.mesh.area / self.k0.real

    def aug_operator(self):
        """Exterior part of eq. sys without the GIBC term, continuity rows
        weighted: [[j k0 A0, -Dv^T Gam], W [Dv, j k0 I]] (what the library's
        augmented product computes)."""
        k0 = self.k0
        W = self.row_weight[:, None]
        top = np.hstack([1j * k0 * self.A0, -self.Dv.T @ self.Gam0])
        bot = W * np.hstack([self.Dv.astype(np.complex128), 1j * k0 * np.eye(self.T)])
        return np.vstack([top, bot])

    def aug_matrix(self):
        """eq. sys with v = Z u eliminated (unknowns u, sigma)."""
        M = self.aug_operator()
        E = self.mesh.nrwg
        M[:E, :E] -= (self.K0 - 0.5 * self.X) @ self.Z() / self.eta0
        return M

    def aug_block_matrix(self):
        """Unnested form over (u, sigma, v): the exterior rows of eq. sys with
        v kept, and the interior equation -(K_i + X/2) u - j w eps~ L_i v = 0
        (eq. MFIE1dis)."""
        E, T = self.mesh.nrwg, self.T
        M = np.zeros((2 * E + T, 2 * E + T), np.complex128)
        M[:E + T, :E + T] = self.aug_operator()
        M[:E, E + T:] = -(self.K0 - 0.5 * self.X) / self.eta0
        M[E + T:, :E] = -(self.Ki + 0.5 * self.X)
        M[E + T:, E + T:] = -1j * self.w * self.eps_vec[:, None] * self.Li
        return M

    def aug_rhs(self, e):
        return np.concatenate([np.asarray(e) / self.eta0, np.zeros(self.T, np.complex128)])

    def solve_aug(self, e):
        """(u, sigma) of eq. sys and v = Z u; the blocks differ in scale by
        many orders at low frequency, so the dense solve is equilibrated
        (rows, then columns, scaled to unit maximum)."""
        E = self.mesh.nrwg
        x = equilibrated_solve(self.aug_matrix(), self.aug_rhs(e))
        u, sg = x[:E], x[E:]
        return u, sg, self.Z() @ u

    def constraint_preconditioner(self):
        """Dense P of the constraint preconditioner (module docstring), with
        the continuity rows weighted like the operator's."""
        k0 = self.k0
        W = self.row_weight[:, None]
        Ad = 1j * k0 * np.diag(np.diag(self.A0))
        B = -self.Dv.T * np.diag(self.Gam0)[None, :]
        top = np.hstack([Ad, B])
        bot = W * np.hstack([self.Dv.astype(np.complex128), 1j * k0 * np.eye(self.T)])
        return np.vstack([top, bot])

    def apply_preconditioner(self, r):
        """P^-1 r through the Schur complement (block elimination of P)."""
        E = self.mesh.nrwg
        k0 = self.k0
        ad = 1j * k0 * np.diag(self.A0)
        gam = np.diag(self.Gam0)
        r1, r2 = r[:E], r[E:] / self.row_weight
        ys = np.linalg.solve(self.schur(), r2 - self.Dv @ (r1 / ad))
        yu = (r1 + self.Dv.T @ (gam * ys)) / ad
        return np.concatenate([yu, ys])

    def schur(self):
        """S = j k0 I - Dv (j k0 diag(A0))^-1 (-Dv^T diag(Gam))."""
        k0 = self.k0
        w = 1.0 / (1j * k0 * np.diag(self.A0))
        return 1j * k0 * np.eye(self.T) + (self.Dv * w[None, :]) @ self.Dv.T * np.diag(self.Gam0)[None, :]


class AugmentedAIM:
    """AIM form of the exterior rows of eq. sys (the library's augmented
    product): the vector potential A0 of an AIMOperator (its precorrected near
    matrix NA plus grid part), and the pulse-charge potential Gam0 through the
    same grid: pulse charges project with the triangle moments M0 (the scalar
    stencil weights without the RWG divergence), the convolved potential is
    tested with M0 per triangle, and the near pairs of the operator carry the
    direct pulse integrals minus their grid part (eq. LinNRP applied to
    pulses)."""

    def __init__(self, op, rules=None):
        self.op = op
        mesh = op.mesh
        self.mesh = mesh
        self.k0 = op.k
        self.T = len(mesh.tri)
        self.Dv = divergence_matrix(mesh)
        div0 = mesh.tri_sign[:, 0] * mesh.tri_len[:, 0] / mesh.area
        tl, sl = op.near_t, op.near_s
        G = np.zeros((self.T, self.T), np.complex128)
        for c0 in range(0, len(tl), 20000):
            a, b = tl[c0:c0 + 20000], sl[c0:c0 + 20000]
            _, ph, _ = pair_blocks(mesh, op.k, a, b, rules)
            direct = ph[:, 0, 0] / (div0[a] * div0[b])
            if op.local:
                grid = 0.0
            else:
                if not hasattr(op, "_Gt"):
                    op._offset_tables()
                dn = op.nodes[a][:, :, None, :] - op.nodes[b][:, None, :, :] + op._W
                Gg = op._Gt[dn[..., 0], dn[..., 1], dn[..., 2]]                    # [P,27,27]
                grid = np.einsum("pa,pab,pb->p", op.M0[a], Gg, op.M0[b])
            G[a, b] += direct - grid
        self.NG = G

    def pulse_far(self, sg):
        """Grid part of Gam0 sigma per triangle: project sigma_t M0_t, convolve
        with G, test with M0_t."""
        op = self.op
        if op.local:
            return np.zeros(self.T, np.complex128)
        n = op.grid.n
        Q = np.zeros((n[2], n[1], n[0]), np.complex128)
        idx = op.nodes
        np.add.at(Q, (idx[..., 2], idx[..., 1], idx[..., 0]), sg[:, None] * op.M0)
        F = op.convolve_fft(Q, "G")
        return np.einsum("ta,ta->t", op.M0, F[idx[..., 2], idx[..., 1], idx[..., 0]])

    def matvec(self, x):
        """[j k0 A0 u - Dv^T Gam0 sigma ; W (Dv u + j k0 sigma)] for x = [u; sigma]."""
        E = self.mesh.nrwg
        u, sg = x[:E], x[E:]
        k0 = self.k0
        yu = 1j * k0 * self.op.matvec(u, "A") - self.Dv.T @ (self.NG @ sg + self.pulse_far(sg))
        W = self.mesh.area / k0.real
        ys = W * (self.Dv @ u + 1j * k0 * sg)
        return np.concatenate([yu, ys])
