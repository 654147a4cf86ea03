"""Mie series for a homogeneous sphere (closed-form pin of the whole path).

TEST INFRASTRUCTURE ONLY.  Coefficients a_n, b_n in the Riccati-Bessel form
of Bohren and Huffman (1983), Ch. 4, with the logarithmic derivative
D_n(m x) from downward recurrence; time dependence e^{-i omega t}, non-
magnetic sphere of radius a in vacuum, relative index m = sqrt(eps_r).
"""
from __future__ import annotations

import numpy as np


def mie_ab(x: float, m: complex, nstop: int | None = None):
    m = complex(m)
    if nstop is None:
        nstop = int(x + 4.0 * x ** (1.0 / 3.0) + 2.0) + 4
    y = m * x
    nmx = int(max(nstop, abs(y))) + 16
    D = np.zeros(nmx + 1, dtype=np.complex128)
    for n in range(nmx, 0, -1):
        D[n - 1] = n / y - 1.0 / (D[n] + n / y)
    psi_m2, psi_m1 = np.cos(x), np.sin(x)      # psi_{-1}, psi_0
    chi_m2, chi_m1 = -np.sin(x), np.cos(x)     # chi_{-1}, chi_0
    a = np.zeros(nstop, dtype=np.complex128)
    b = np.zeros(nstop, dtype=np.complex128)
    xi_m1 = psi_m1 - 1j * chi_m1
    for n in range(1, nstop + 1):
        psi = (2 * n - 1) / x * psi_m1 - psi_m2
        chi = (2 * n - 1) / x * chi_m1 - chi_m2
        xi = psi - 1j * chi
        ta = D[n] / m + n / x
        tb = m * D[n] + n / x
        a[n - 1] = (ta * psi - psi_m1) / (ta * xi - xi_m1)
        b[n - 1] = (tb * psi - psi_m1) / (tb * xi - xi_m1)
        psi_m2, psi_m1 = psi_m1, psi
        chi_m2, chi_m1 = chi_m1, chi
        xi_m1 = xi
    return a, b


def cross_sections(k: float, radius: float, eps_r: complex):
    """(C_ext, C_sca, C_abs) for unit-amplitude incidence."""
    x = k * radius
    a, b = mie_ab(x, np.sqrt(complex(eps_r)))
    n = np.arange(1, a.shape[0] + 1)
    qext = 2.0 / x ** 2 * np.sum((2 * n + 1) * np.real(a + b))
    qsca = 2.0 / x ** 2 * np.sum((2 * n + 1) * (np.abs(a) ** 2 + np.abs(b) ** 2))
    g = np.pi * radius ** 2
    return qext * g, qsca * g, (qext - qsca) * g


def amplitudes(k: float, radius: float, eps_r: complex, theta):
    """S1(theta), S2(theta) (Bohren and Huffman eq. 4.74 notation)."""
    a, b = mie_ab(k * radius, np.sqrt(complex(eps_r)))
    theta = np.atleast_1d(theta)
    mu = np.cos(theta)
    S1 = np.zeros(theta.shape, dtype=np.complex128)
    S2 = np.zeros_like(S1)
    pi_m1 = np.zeros_like(mu)
    pi_n = np.ones_like(mu)
    for n in range(1, a.shape[0] + 1):
        tau = n * mu * pi_n - (n + 1) * pi_m1
        f = (2 * n + 1) / (n * (n + 1))
        S1 += f * (a[n - 1] * pi_n + b[n - 1] * tau)
        S2 += f * (a[n - 1] * tau + b[n - 1] * pi_n)
        pi_next = ((2 * n + 1) * mu * pi_n - (n + 1) * pi_m1) / n
        pi_m1, pi_n = pi_n, pi_next
    return S1, S2


def far_field(k: float, radius: float, eps_r: complex, rhat):
    """F(r) for incidence along +z polarised along +x, E_s ~ F e^{ikr}/r."""
    rhat = np.atleast_2d(rhat)
    th = np.arccos(np.clip(rhat[:, 2], -1, 1))
    ph = np.arctan2(rhat[:, 1], rhat[:, 0])
    S1, S2 = amplitudes(k, radius, eps_r, th)
    eth = np.stack([np.cos(th) * np.cos(ph), np.cos(th) * np.sin(ph), -np.sin(th)], 1)
    eph = np.stack([-np.sin(ph), np.cos(ph), np.zeros_like(ph)], 1)
    return (1j / k) * ((np.cos(ph) * S2)[:, None] * eth - (np.sin(ph) * S1)[:, None] * eph)
