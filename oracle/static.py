"""Closed-form static potentials of a flat triangle (singularity extraction).

The paper only says that near-region entries are found by accurate direct
integration (Sec. III-D-1) and cites "advanced" techniques for lossy media
(Sec. V-C).  The oracle extracts the 1/R part of G and integrates it in closed
form (Wilton et al., IEEE TAP 1984; Graglia, IEEE TAP 1993):

  I(r)      = int_T 1/R dS'
  Irho(r)   = int_T (rho' - rho)/R dS'       (rho = projection of r on the plane)
  gradI(r)  = grad_r int_T 1/R dS'

For each edge i (vertex a -> b, counter-clockwise), with unit edge vector l,
outward in-plane edge normal m = l x n, height d = n.(r - v0),
l+/- = (b/a - r).l, t = (a - r).m, R+/- = |r - b/a|, R0^2 = t^2 + d^2:

  f_i    = ln((R+ + l+)/(R- + l-))
  beta_i = atan(t l+/(R0^2 + |d| R+)) - atan(t l-/(R0^2 + |d| R-))
  I      = sum t f - |d| sum beta
  Irho   = 1/2 sum m (R0^2 f + l+ R+ - l- R-)
  gradI  = -sum m f - n sign(d) sum beta

For observation points in the plane of the triangle (|d| below 1e-10 of an
edge length) sign(d) is taken as 0: the in-plane principal value.
"""
import numpy as np


def _log_ratio(lp, lm, Rp, Rm, R02):
    """ln((R+ + l+)/(R- + l-)) in a cancellation-free form for every position of
    the foot point relative to the edge segment."""
    tiny = np.finfo(np.float64).tiny
    both_pos = lm >= 0.0
    both_neg = lp <= 0.0
    mixed = ~(both_pos | both_neg)
    f = np.zeros_like(lp)
    with np.errstate(divide="ignore", invalid="ignore"):
        f1 = np.log(np.maximum(Rp + lp, tiny) / np.maximum(Rm + lm, tiny))
        f2 = np.log(np.maximum(Rm - lm, tiny) / np.maximum(Rp - lp, tiny))
        f3 = np.log(np.maximum((Rp + lp) * (Rm - lm), tiny)) - np.log(np.maximum(R02, tiny))
    f = np.where(both_pos, f1, f)
    f = np.where(both_neg, f2, f)
    f = np.where(mixed, f3, f)
    return f


def triangle_potentials(verts, obs):
    """verts [P,3,3], obs [P,Q,3] -> (I [P,Q], Irho [P,Q,3], gradI [P,Q,3])."""
    verts = np.asarray(verts, dtype=np.float64)
    obs = np.asarray(obs, dtype=np.float64)
    v0, v1, v2 = verts[:, 0], verts[:, 1], verts[:, 2]
    n = np.cross(v1 - v0, v2 - v0)
    n /= np.linalg.norm(n, axis=1)[:, None]
    d = np.einsum("pqc,pc->pq", obs - v0[:, None, :], n)
    # points in the source plane up to rounding take the principal value
    d = np.where(np.abs(d) <= 1e-10 * np.linalg.norm(v1 - v0, axis=1)[:, None], 0.0, d)
    absd = np.abs(d)
    I = np.zeros(obs.shape[:2])
    Irho = np.zeros(obs.shape)
    gI = np.zeros(obs.shape)
    sb = np.zeros(obs.shape[:2])
    for i in range(3):
        a = verts[:, i]
        b = verts[:, (i + 1) % 3]
        le = b - a
        lhat = le / np.linalg.norm(le, axis=1)[:, None]
        mhat = np.cross(lhat, n)
        lp = np.einsum("pqc,pc->pq", b[:, None, :] - obs, lhat)
        lm = np.einsum("pqc,pc->pq", a[:, None, :] - obs, lhat)
        t = np.einsum("pqc,pc->pq", a[:, None, :] - obs, mhat)
        Rp = np.linalg.norm(obs - b[:, None, :], axis=2)
        Rm = np.linalg.norm(obs - a[:, None, :], axis=2)
        R02 = t * t + d * d
        f = _log_ratio(lp, lm, Rp, Rm, R02)
        with np.errstate(divide="ignore", invalid="ignore"):
            beta = (np.arctan2(t * lp, R02 + absd * Rp) - np.arctan2(t * lm, R02 + absd * Rm))
        online = R02 <= 1e-30 * (lp * lp + lm * lm + 1e-300)
        beta = np.where(online, 0.0, beta)
        tf = np.where(online, 0.0, t * f)
        I += tf
        sb += beta
        coef = np.where(online, 0.0, R02 * f) + lp * Rp - lm * Rm
        Irho += 0.5 * coef[..., None] * mhat[:, None, :]
        gI -= f[..., None] * mhat[:, None, :]
    I -= absd * sb
    gI -= (np.sign(d) * sb)[..., None] * n[:, None, :]
    return I, Irho, gI
