"""Dense solves of the GIBC system (Sec. III-A to III-C).

Unknowns per object: u = n x H and v = n x E (RWG coefficients, n outward).
Derived from the surface equivalence principle with e^{j omega t}, the
Galerkin-tested equations are

  exterior (EFIE, eq. EFIE01dis):  j w mu0 L0 u - (K0 - X/2) v = e
  interior (MFIE, eq. MFIE1dis):   -j w eps~_i L_i v - (K_i + X/2) u = 0

The printed half-terms, -(K_i - X/2) and -(K0 + X/2) with right-hand side
-E_inc, describe the same physics when K is written with the source-point
gradient and the exterior unknown is n0 x H = -u (n0 = -n_i); the form above is
the one used throughout, and the Mie series pins its signs.

GIBC (eq. GIBCdef, GIBCsys): v_i = Z_i u_i with
  Z_i = -(j w eps~_i)^-1 L_i^-1 (K_i + X/2),
  [j w mu0 L0 - (K0 - X/2) Z] u = e.
"""
import numpy as np

from . import physics as ph
from .mom import dense_operators, L_from, x_matrix, excitation


class DenseProblem:
    """All dense matrices of a problem (exterior at k0; interior per object)."""

    def __init__(self, mesh, freq, materials, bg_eps_r=1.0, bg_mu_r=1.0, rules=None):
        self.mesh = mesh
        self.freq = freq
        self.w = ph.omega(freq)
        self.k0 = ph.wavenumber(freq, bg_eps_r, bg_mu_r, 0.0)
        self.eps0 = ph.EPS0 * bg_eps_r
        self.mu0 = ph.MU0 * bg_mu_r
        self.eta0 = np.sqrt(self.mu0 / self.eps0)
        A0, P0, K0 = dense_operators(mesh, self.k0, rules=rules)
        self.A0, self.P0, self.K0 = A0, P0, K0
        self.L0 = L_from(A0, P0, self.k0)
        self.X = x_matrix(mesh)
        E = mesh.nrwg
        self.Li = np.zeros((E, E), np.complex128)
        self.Ki = np.zeros((E, E), np.complex128)
        self.ki = []
        self.epst = []
        self.obj_rng = []
        for i, (eps_r, mu_r, sigma) in enumerate(materials):
            ki = ph.wavenumber(freq, eps_r, mu_r, sigma)
            et = ph.eps_tilde(freq, eps_r, sigma)
            a, b = mesh.obj_rwg_range(i)
            Ai, Pi, Ki = dense_operators(mesh, ki, obj=i, rules=rules)
            sl = slice(a, b)
            self.Li[sl, sl] = L_from(Ai, Pi, ki)[sl, sl]
            self.Ki[sl, sl] = Ki[sl, sl]
            self.ki.append(ki)
            self.epst.append(et)
            self.obj_rng.append((a, b))
        eps_vec = np.zeros(E, np.complex128)
        for (a, b), et in zip(self.obj_rng, self.epst):
            eps_vec[a:b] = et
        self.eps_vec = eps_vec

    def rhs(self, khat, e0):
        return excitation(self.mesh, self.k0, khat, e0)

    def block_matrix(self):
        """[[j w mu0 L0, -(K0 - X/2)], [-(Ki + X/2), -j w eps~ Li]]."""
        w = self.w
        top = np.hstack([1j * w * self.mu0 * self.L0, -(self.K0 - 0.5 * self.X)])
        bot = np.hstack([-(self.Ki + 0.5 * self.X), -1j * w * self.eps_vec[:, None] * self.Li])
        return np.vstack([top, bot])

    def solve_block(self, e):
        E = self.mesh.nrwg
        x = np.linalg.solve(self.block_matrix(), np.concatenate([e, np.zeros(E, np.complex128)]))
        return x[:E], x[E:]

    def Z(self):
        """Block-diagonal GIBC operator Z = -(j w eps~)^-1 Li^-1 (Ki + X/2)."""
        E = self.mesh.nrwg
        Z = np.zeros((E, E), np.complex128)
        for (a, b), et in zip(self.obj_rng, self.epst):
            sl = slice(a, b)
            Z[sl, sl] = -np.linalg.solve(1j * self.w * et * self.Li[sl, sl],
                                         self.Ki[sl, sl] + 0.5 * self.X[sl, sl])
        return Z

    def gibc_matrix(self):
        return 1j * self.w * self.mu0 * self.L0 - (self.K0 - 0.5 * self.X) @ self.Z()

    def solve_gibc(self, e):
        Z = self.Z()
        u = np.linalg.solve(1j * self.w * self.mu0 * self.L0 - (self.K0 - 0.5 * self.X) @ Z, e)
        return u, Z @ u
