"""Pins of the oracle's derivatives (central differences with Richardson
extrapolation of the whole discrete map).

* The kernel-difference derivatives with respect to eps_r match the
  textbook derivatives of the Helmholtz kernel, e.g. d phi/dk = i R phi for
  phi = e^{ikR}/(4 pi R), through k_i = k0 sqrt(eps_r) (dk_i/deps_r =
  k_i / (2 eps_r)), on both sides of the series/closed-form switch.
* The differences converge (step h and h/2 agree).
* s(eps) = conj(e).F(khat) is holomorphic in eps_r: its derivatives along
  Re and Im eps_r satisfy ds/dIm = i ds/dRe (Cauchy-Riemann), which fixes
  how sigma_ext = (4 pi/k) Im s turns a complex derivative into the two
  real ones.
"""
import numpy as np

from oracle import adjoint, core, galerkin
from workloads import icosphere_p2

KH = np.array([0.0, 0.0, 1.0])
POL = np.array([1.0, 0.0, 0.0], dtype=np.complex128)


def test_kernel_scalar_derivatives_closed_forms():
    k0, eps = 3.0, 3.0 + 0.1j
    ki = k0 * np.sqrt(eps)
    dk = ki / (2 * eps)
    R = np.array([0.02, 0.1, 0.3, 0.9])     # series and closed-form branches
    d = adjoint.richardson(lambda e: np.stack(core.kernel_scalars(core.phys_vector(k0, e), R)),
                           eps, 1e-4)
    e = np.exp(1j * ki * R)
    phi = e / (4 * np.pi * R)
    dphi = 1j * R * phi
    dD0 = -(2 * ki * phi + ki ** 2 * dphi) * dk                # D0 = ka^2 phi_a - ki^2 phi_i
    dg = e * ki / (4 * np.pi * R)                              # g = e (1 - ikR) / (4 pi R^3)
    df = e * ki * (1 - 1j * ki * R) / (4 * np.pi * R)          # f = e (3 - 3ikR - k^2R^2)/(4 pi R^3)
    g = e * (1 - 1j * ki * R) / (4 * np.pi * R ** 3)
    dGe = R * (g + eps * dg * dk)                              # G_eps = -R (g_a - eps g_i)
    for got, ref in ((d[0], dD0), (d[1], -df * dk), (d[2], -dg * dk), (d[3], dGe)):
        assert np.abs(got - ref).max() < 1e-7 * np.abs(ref).max()


def test_dsigma_differences_converge():
    xyz, tri = icosphere_p2(80)
    a = adjoint.dsigma_deps(xyz, tri, 3.0, 3.0 + 0.1j, KH, POL, h=1e-3)
    b = adjoint.dsigma_deps(xyz, tri, 3.0, 3.0 + 0.1j, KH, POL, h=5e-4)
    for u, v in zip(a, b):
        assert abs(u - v) < 1e-8 * max(abs(u), abs(v))


def test_far_field_functional_is_holomorphic_in_eps():
    xyz, tri = icosphere_p2(80)

    def s(e):
        _, x, _, P = adjoint.solve_sigma_ext(xyz, tri, 2.0, e, KH, POL)
        return np.vdot(POL, galerkin.far_field(P, x, KH[None])[0])

    eps = 4.0 + 0.3j
    d_re = adjoint.richardson(lambda t: s(eps + t), 0.0, 1e-3)
    d_im = adjoint.richardson(lambda t: s(eps + 1j * t), 0.0, 1e-3)
    assert abs(d_im - 1j * d_re) < 1e-8 * abs(d_re)
