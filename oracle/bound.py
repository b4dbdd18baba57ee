"""Interpolation error bound of the AIM for lossy media (Sec. IV).

Loss factor s = sigma/(omega eps_i), k = k_r sqrt(1 - j s) (eq. kdefs), lengths
normalised as theta = k_r d.  The (n+1)-th derivative of exp(-j theta a)/theta,
a = sqrt(1 - j s), written out with the product rule (eq. Ddef):

  D_n(theta, s) = exp(-j theta a) sum_{l=0}^{n+1} C(n+1, l) (-1)^(n+1-l)
                  (n+1-l)! theta^-(n-l+2) (-j a)^l

and the bound (eq. LboundsD2), with |D_n| decreasing in theta:

  Delta G_n / k_r <= (theta_n - theta_0)^(n+1)/(n+1)! |D_n(theta_0, s)|
"""
import math

import numpy as np


def D(n, theta, s):
    a = np.sqrt(1.0 - 1j * np.asarray(s, dtype=np.float64))
    theta = np.asarray(theta, dtype=np.float64)
    acc = 0.0
    for l in range(n + 2):
        acc = acc + (math.comb(n + 1, l) * (-1.0) ** (n + 1 - l) * math.factorial(n + 1 - l)
                     * theta ** (-(n - l + 2)) * (-1j * a) ** l)
    return np.exp(-1j * theta * a) * acc


def bound(n, theta0, thetan, s):
    """Right-hand side of eq. LboundsD2 (Delta G_n / k_r)."""
    return (thetan - theta0) ** (n + 1) / math.factorial(n + 1) * np.abs(D(n, theta0, s))


def loss_ratio(n, theta0, s):
    """Delta G_n / Delta G_n,lossless for the same grid: |D_n(theta0,s)|/|D_n(theta0,0)|."""
    return np.abs(D(n, theta0, s)) / np.abs(D(n, theta0, 0.0))


def worst_loss_ratio(n, theta=(0.05, 20.0, 2001), s=(-4.0, 6.0, 2001)):
    """Maximum of loss_ratio over a log-spaced (theta0, s) window, refined once
    around the coarse maximum.  Returns (ratio, theta0, s)."""
    th = np.geomspace(theta[0], theta[1], theta[2])
    ss = np.logspace(s[0], s[1], s[2])
    R = loss_ratio(n, th[:, None], ss[None, :])
    i, j = np.unravel_index(np.nanargmax(R), R.shape)
    th2 = np.linspace(th[max(i - 2, 0)], th[min(i + 2, len(th) - 1)], 401)
    ss2 = np.linspace(ss[max(j - 2, 0)], ss[min(j + 2, len(ss) - 1)], 401)
    R2 = loss_ratio(n, th2[:, None], ss2[None, :])
    i2, j2 = np.unravel_index(np.nanargmax(R2), R2.shape)
    return R2[i2, j2], th2[i2], ss2[j2]
