"""Self-consistency pins of the Mie series oracle."""
import numpy as np

from oracle import mie


def test_extinction_equals_scattering_lossless():
    ce, cs = mie.cross_sections(3.0, 1.0, 4.0)
    assert abs(ce - cs) < 1e-12 * cs


def test_integrated_bistatic_equals_csca():
    k, eps = 2.0, 3.0 - 1.0j
    _, cs = mie.cross_sections(k, 1.0, eps)
    th = np.linspace(0, np.pi, 3001); phs = np.linspace(0, 2 * np.pi, 32, endpoint=False)
    TH, PH = np.meshgrid(th, phs, indexing="ij")
    r = mie.bistatic_rcs(k, 1.0, eps, TH, PH)
    integ = np.trapezoid(r.mean(axis=1) * np.sin(th), th) * 2 * np.pi / (4 * np.pi)
    assert abs(integ - cs) < 1e-5 * cs


def test_rayleigh_limit():
    """Small sphere: C_sca = (8 pi/3) k^4 a^6 |(m^2-1)/(m^2+2)|^2."""
    k, a, eps = 1e-2, 1.0, 4.0
    _, cs = mie.cross_sections(k, a, eps)
    ray = 8 * np.pi / 3 * k ** 4 * a ** 6 * abs((eps - 1) / (eps + 2)) ** 2
    assert abs(cs - ray) < 1e-3 * ray


def test_absorption_positive_for_lossy():
    ce, cs = mie.cross_sections(2.0, 1.0, 4.0 - 2.0j)
    assert ce > cs > 0
