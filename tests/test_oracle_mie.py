"""Pins of the Mie series used as the sphere closed form."""
import numpy as np
import pytest
from scipy.special import spherical_jn, spherical_yn

from oracle import mie


def _ab_direct(x, m, nmax):
    """a_n, b_n straight from the Riccati-Bessel definitions with scipy's
    spherical Bessel functions (real m, no recurrences of our own)."""
    n = np.arange(1, nmax + 1)
    mx = m * x

    def psi(n, z):
        return z * spherical_jn(n, z)

    def dpsi(n, z):
        return spherical_jn(n, z) + z * spherical_jn(n, z, derivative=True)

    def xi(n, z):
        return z * (spherical_jn(n, z) + 1j * spherical_yn(n, z))

    def dxi(n, z):
        return (spherical_jn(n, z) + 1j * spherical_yn(n, z)) + z * (
            spherical_jn(n, z, derivative=True) + 1j * spherical_yn(n, z, derivative=True))

    a = (m * psi(n, mx) * dpsi(n, x) - psi(n, x) * dpsi(n, mx)) / (
        m * psi(n, mx) * dxi(n, x) - xi(n, x) * dpsi(n, mx))
    b = (psi(n, mx) * dpsi(n, x) - m * psi(n, x) * dpsi(n, mx)) / (
        psi(n, mx) * dxi(n, x) - m * xi(n, x) * dpsi(n, mx))
    return a, b


@pytest.mark.parametrize("x,eps", [(1.0, 4.0), (5.0, 2.25), (3.0, 6.0)])
def test_coefficients_match_scipy(x, eps):
    a, b = mie.mie_ab(x, np.sqrt(eps))
    a2, b2 = _ab_direct(x, np.sqrt(eps), a.shape[0])
    assert np.abs(a - a2).max() < 1e-12
    assert np.abs(b - b2).max() < 1e-12


@pytest.mark.parametrize("x,eps", [(1.0, 4.0), (5.0, 2.25), (3.0, 6.0)])
def test_lossless_energy_balance(x, eps):
    ce, cs, ca = mie.cross_sections(x, 1.0, eps)
    assert abs(ca) < 1e-12 * ce


def test_rayleigh_limit():
    """Small spheres: Q_sca -> (8/3) x^4 |(m^2-1)/(m^2+2)|^2."""
    x, eps = 1e-3, 3.0 + 0.5j
    ce, cs, ca = mie.cross_sections(x, 1.0, eps)
    q = cs / np.pi
    ref = 8.0 / 3.0 * x ** 4 * abs((eps - 1) / (eps + 2)) ** 2
    assert abs(q - ref) / ref < 1e-5
    # absorption dominates: Q_abs -> 4 x Im((m^2-1)/(m^2+2))
    qa = ca / np.pi
    assert abs(qa - 4 * x * np.imag((eps - 1) / (eps + 2))) / qa < 1e-5


def test_forward_amplitude_optical_theorem():
    """C_ext = (4 pi / k) Im(x . F(z)) with the far-field convention used
    by the oracle (F = (i/k)(cos phi S2 e_th - sin phi S1 e_ph))."""
    k, eps = 5.0, 2.25
    ce, cs, ca = mie.cross_sections(k, 1.0, eps)
    F = mie.far_field(k, 1.0, eps, np.array([[0.0, 0.0, 1.0]]))[0]
    assert abs(4 * np.pi / k * F[0].imag - ce) < 1e-12 * ce


def test_scattered_power_integral():
    """int |F|^2 dOmega = C_sca."""
    from oracle.galerkin import sphere_quadrature
    k, eps = 3.0, 6.0
    _, cs, _ = mie.cross_sections(k, 1.0, eps)
    d, w = sphere_quadrature(40)
    F = mie.far_field(k, 1.0, eps, d)
    assert abs(np.sum(w * np.sum(np.abs(F) ** 2, 1)) - cs) < 1e-10 * cs
