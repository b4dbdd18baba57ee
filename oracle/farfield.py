"""Scattered far field and radar cross section (Sec. V-A).

With J = u = n x H and M = -v = E x n on S radiating in the background medium,

  E_s(r rhat) ~ exp(-j k0 r)/(4 pi r) (-j k0) [eta0 (N_u - rhat (rhat . N_u)) + rhat x N_v]
  N_x = int x(r') exp(j k0 rhat . r') dS'
  RCS = 4 pi r^2 |E_s|^2 / |E_inc|^2
"""
import numpy as np

from .quad import collapsed_gauss, points_on


def radiation_vectors(mesh, k0, coef, rhat, n_q=6):
    """N = int sum_n coef_n f_n(r') exp(j k0 rhat . r') dS' for rhat [D,3]."""
    bary, w = collapsed_gauss(n_q)
    pts = points_on(mesh.verts, bary)                    # [T,Q,3]
    c = mesh.tri_sign * mesh.tri_len / (2.0 * mesh.area)[:, None]
    f = c[:, None, :, None] * (pts[:, :, None, :] - mesh.verts[:, None, :, :])   # [T,Q,3,3]
    x = coef[mesh.tri_rwg]                               # [T,3]
    cur = np.einsum("te,tqec->tqc", x, f)                # [T,Q,3]
    ph = np.exp(1j * k0 * np.einsum("dc,tqc->dtq", rhat, pts))
    return np.einsum("dtq,tqc,q,t->dc", ph, cur, w, mesh.area)


def far_field(mesh, k0, eta0, u, v, rhat):
    """Complex far-field amplitude F with E_s ~ F exp(-j k0 r)/r: [D,3]."""
    rhat = np.asarray(rhat, dtype=np.float64)
    Nu = radiation_vectors(mesh, k0, u, rhat)
    Nv = radiation_vectors(mesh, k0, v, rhat)
    Nu_t = Nu - rhat * np.einsum("dc,dc->d", rhat, Nu)[:, None]
    return (-1j * k0 / (4.0 * np.pi)) * (eta0 * Nu_t + np.cross(rhat, Nv))


def rcs(mesh, k0, eta0, u, v, rhat):
    F = far_field(mesh, k0, eta0, u, v, rhat)
    return 4.0 * np.pi * np.sum(np.abs(F) ** 2, axis=1)


def directions(theta, phi):
    theta = np.asarray(theta, float); phi = np.asarray(phi, float)
    return np.stack([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi), np.cos(theta)], axis=-1)
