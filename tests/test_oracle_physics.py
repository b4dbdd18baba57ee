"""Material constants of the oracle (Sec. II, eq. kin and eq. etain) against
textbook closed forms that do not go through the same square roots."""
import numpy as np

from oracle import physics as ph


def test_free_space_impedance():
    # eta0 = mu0 c0 with mu0 = 4 pi 1e-7 H/m and c0 = 299,792,458 m/s
    assert abs(ph.impedance(1e9, 1.0) - 376.730313461) < 1e-6
    # lossless dielectric: eta0 / sqrt(eps_r); frequency-independent
    assert abs(ph.impedance(3e8, 4.0) - 376.730313461 / 2.0) < 1e-6


def test_good_conductor_skin_depth_and_surface_impedance():
    # copper at 10 GHz: delta = sqrt(2 / (w mu0 sigma)) = 0.661 um and the
    # surface impedance (1 + j) / (sigma delta) (e^{+jwt}: inductive), both to
    # first order in w eps0 / sigma ~ 1e-8
    f, s = 10e9, 5.8e7
    delta = np.sqrt(2.0 / (2 * np.pi * f * 4e-7 * np.pi * s))
    assert abs(delta - 0.6608549e-6) < 1e-12
    k = ph.wavenumber(f, 1.0, 1.0, s)
    assert abs(ph.skin_depth(k) / delta - 1.0) < 1e-7
    eta = ph.impedance(f, 1.0, 1.0, s)
    assert abs(eta / ((1 + 1j) / (s * delta)) - 1.0) < 1e-7


def test_skin_depth_lossless_is_infinite():
    assert ph.skin_depth(ph.wavenumber(1e9, 4.0)) == np.inf


def test_lossy_wavenumber_decays_and_matches_low_loss_expansion():
    # low loss s = sigma / (w eps) << 1: k ~ k_r (1 - j s / 2)
    f, er, s = 1e9, 4.0, 1e-4
    w = 2 * np.pi * f
    sigma = s * w * ph.EPS0 * er
    k = ph.wavenumber(f, er, 1.0, sigma)
    kr = w * np.sqrt(er) / ph.C0
    assert k.imag < 0
    assert abs(k - kr * (1 - 0.5j * s)) < 1e-7 * kr
