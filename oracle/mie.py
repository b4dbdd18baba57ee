"""Mie series for a homogeneous sphere (the analytic reference of Sec. V-A).

Bohren & Huffman (1983), ch. 4, with the logarithmic-derivative recurrence
D_n(m x) computed downwards and n_max = x + 4 x^(1/3) + 2 (Wiscombe).  Their
time convention is e^{-i w t}: a lossy sphere of complex permittivity
eps~ = eps0 eps_r - j sigma/w (e^{+j w t}) has relative index m = conj(sqrt(eps~/eps0)).
Intensities (RCS, cross sections) do not depend on the convention.
"""
import numpy as np


def _coefficients(x, m):
    nmax = int(np.round(x + 4.0 * x ** (1.0 / 3.0) + 2.0))
    mx = m * x
    nmx = int(np.round(max(nmax, abs(mx)) + 16))
    D = np.zeros(nmx + 1, np.complex128)
    for n in range(nmx, 0, -1):
        D[n - 1] = n / mx - 1.0 / (D[n] + n / mx)
    psi0, psi1 = np.cos(x), np.sin(x)          # psi_{-1}, psi_0
    chi0, chi1 = -np.sin(x), np.cos(x)
    xi1 = psi1 - 1j * chi1
    a = np.zeros(nmax, np.complex128)
    b = np.zeros(nmax, np.complex128)
    for n in range(1, nmax + 1):
        psi = (2 * n - 1) / x * psi1 - psi0
        chi = (2 * n - 1) / x * chi1 - chi0
        xi = psi - 1j * chi
        a[n - 1] = ((D[n] / m + n / x) * psi - psi1) / ((D[n] / m + n / x) * xi - xi1)
        b[n - 1] = ((m * D[n] + n / x) * psi - psi1) / ((m * D[n] + n / x) * xi - xi1)
        psi0, psi1 = psi1, psi
        chi0, chi1 = chi1, chi
        xi1 = psi1 - 1j * chi1
    return a, b


def coefficients(k0, radius, eps_tilde_rel):
    """(a_n, b_n) for size parameter x = k0 a and index m = conj(sqrt(eps~_r))."""
    m = np.conj(np.sqrt(complex(eps_tilde_rel)))
    if m.real < 0:
        m = -m
    x = float(np.real(k0)) * radius
    return _coefficients(x, m)


def amplitudes(a, b, theta):
    """S1(theta), S2(theta) (Bohren & Huffman eq. 4.74)."""
    mu = np.cos(np.asarray(theta, float))
    S1 = np.zeros(mu.shape, np.complex128)
    S2 = np.zeros(mu.shape, np.complex128)
    pi0 = np.zeros_like(mu); pi1 = np.ones_like(mu)
    for n in range(1, len(a) + 1):
        tau = n * mu * pi1 - (n + 1) * pi0
        c = (2 * n + 1) / (n * (n + 1))
        S1 += c * (a[n - 1] * pi1 + b[n - 1] * tau)
        S2 += c * (a[n - 1] * tau + b[n - 1] * pi1)
        pi0, pi1 = pi1, ((2 * n + 1) * mu * pi1 - (n + 1) * pi0) / n
    return S1, S2


def bistatic_rcs(k0, radius, eps_tilde_rel, theta, phi):
    """RCS for an x-polarised wave along +z: 4 pi/k^2 (|S2|^2 cos^2 phi + |S1|^2 sin^2 phi)."""
    k0 = float(np.real(k0))
    a, b = coefficients(k0, radius, eps_tilde_rel)
    S1, S2 = amplitudes(a, b, theta)
    phi = np.asarray(phi, float)
    return 4.0 * np.pi / k0 ** 2 * (np.abs(S2) ** 2 * np.cos(phi) ** 2 + np.abs(S1) ** 2 * np.sin(phi) ** 2)


def cross_sections(k0, radius, eps_tilde_rel):
    """(C_ext, C_sca) from the series (B&H eq. 4.61, 4.62)."""
    k0 = float(np.real(k0))
    a, b = coefficients(k0, radius, eps_tilde_rel)
    n = np.arange(1, len(a) + 1)
    x2 = k0 ** 2
    csca = 2 * np.pi / x2 * np.sum((2 * n + 1) * (np.abs(a) ** 2 + np.abs(b) ** 2))
    cext = 2 * np.pi / x2 * np.sum((2 * n + 1) * (a + b).real)
    return cext, csca
