"""Pins of the Sec. IV error-bound oracle (eq. Ddef, LboundsD2) and its printed
worked value."""
import math
import os

import numpy as np

from oracle.bound import D, bound, loss_ratio, worst_loss_ratio

GOLD = os.path.join(os.path.dirname(__file__), "golden", "bound_worked_example.txt")


def _golden():
    vals = {}
    for line in open(GOLD):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            vals[k] = float(v)
    return vals


def test_printed_worst_case_ratio():
    g = _golden()
    n = int(g["n"])
    # the ratio at the printed point rounds to the printed value
    assert round(float(loss_ratio(n, g["theta0"], g["s"])), 3) == g["ratio"]
    # and the printed point is the maximiser over a wide window
    r, th, s = worst_loss_ratio(n)
    assert abs(r - g["ratio"]) < 5e-4
    assert abs(th - g["theta0"]) < 5e-3
    assert abs(s - g["s"]) / g["s"] < 0.02


def _cauchy_derivative(f, z0, order, radius=0.05, m=256):
    """order-th derivative of an analytic f at z0 by the Cauchy integral formula."""
    t = 2 * np.pi * np.arange(m) / m
    z = z0 + radius * np.exp(1j * t)
    return math.factorial(order) * np.mean(f(z) * np.exp(-1j * order * t)) / radius ** order


def test_D_is_derivative_of_lossy_green():
    for n in range(4):
        for theta, s in ((0.7, 0.0), (1.653, 2.894), (3.0, 50.0), (0.3, 1e-3)):
            a = np.sqrt(1.0 - 1j * s)
            f = lambda th: np.exp(-1j * th * a) / th
            ref = _cauchy_derivative(f, theta, n + 1, radius=0.2 * theta)
            assert abs(D(n, theta, s) - ref) <= 1e-9 * abs(ref)


def test_D_monotone_in_theta():
    th = np.linspace(0.05, 30.0, 3000)
    for s in (0.0, 0.1, 2.894, 100.0):
        d = np.abs(D(2, th, s))
        assert np.all(np.diff(d) < 0)


def test_lagrange_error_below_bound():
    """Actual interpolation error of exp(-j a theta)/theta on n+1 points is below
    the bound of eq. LboundsD2 (lengths normalised by k_r)."""
    for n in (1, 2, 3):
        for s in (0.0, 2.894, 30.0):
            a = np.sqrt(1.0 - 1j * s)
            f = lambda th: np.exp(-1j * th * a) / th
            for th0, span in ((1.0, 0.5), (2.0, 1.0), (0.5, 0.3)):
                nodes = th0 + span * np.arange(n + 1) / n
                x = np.linspace(nodes[0], nodes[-1], 401)
                L = np.zeros_like(x, dtype=complex)
                for q in range(n + 1):
                    lq = np.ones_like(x)
                    for mm in range(n + 1):
                        if mm != q:
                            lq *= (x - nodes[mm]) / (nodes[q] - nodes[mm])
                    L += f(nodes[q]) * lq
                err = np.abs(f(x) - L).max()
                assert err <= bound(n, nodes[0], nodes[-1], s) * (1 + 1e-12)
