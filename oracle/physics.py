"""Material constants (Sec. II, eq. kin and eq. etain).

Time convention e^{+j omega t}.  The complex permittivity folds in the
conductivity, eps~ = eps0*eps_r - j*sigma/omega, and every prefactor that the
paper writes with eps_i uses eps~ (the only reading consistent with eq. kin).
"""
import numpy as np

C0 = 299792458.0
MU0 = 4e-7 * np.pi
EPS0 = 1.0 / (MU0 * C0 * C0)
ETA0 = MU0 * C0


def omega(freq):
    return 2.0 * np.pi * freq


def eps_tilde(freq, eps_r, sigma):
    """eps0*eps_r - j sigma/omega."""
    return EPS0 * eps_r - 1j * sigma / omega(freq)


def wavenumber(freq, eps_r, mu_r=1.0, sigma=0.0):
    """k = sqrt(omega mu (omega eps - j sigma)) (eq. kin), principal branch:
    Re k > 0, Im k <= 0, so exp(-j k r) decays."""
    w = omega(freq)
    k = np.sqrt(complex(w * MU0 * mu_r * (w * EPS0 * eps_r - 1j * sigma)))
    if k.real < 0:
        k = -k
    return k


def impedance(freq, eps_r, mu_r=1.0, sigma=0.0):
    """eta = sqrt(omega mu / (omega eps - j sigma)) (eq. etain)."""
    w = omega(freq)
    eta = np.sqrt(complex(w * MU0 * mu_r / (w * EPS0 * eps_r - 1j * sigma)))
    if eta.real < 0:
        eta = -eta
    return eta


def skin_depth(k):
    """Distance over which |exp(-j k r)| falls by 1/e."""
    return np.inf if k.imag == 0 else -1.0 / k.imag
