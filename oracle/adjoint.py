"""sigma_ext and its derivatives for the adjoint gradient (oracle).

TEST INFRASTRUCTURE ONLY.  The extinction cross section follows the
optical theorem, sigma_ext = (4 pi / k_a) Im(conj(e) . F(khat)), with the
far field of ``galerkin.far_field`` and the solution of the dense system
by LU.  Derivatives are taken by their definition: central differences of
the whole discrete map (fill, assembly, solve, far field) combined by
Richardson extrapolation,
    f'(a) ~ [8 (f(a+h) - f(a-h)) - (f(a+2h) - f(a-2h))] / (12 h),
whose error is O(h^4) plus rounding of order u |f| / h.
"""
from __future__ import annotations

import numpy as np

from . import core, galerkin


def sigma_ext(P, x, khat, pol):
    F = galerkin.far_field(P, x, np.asarray(khat, dtype=np.float64)[None])[0]
    return 4 * np.pi / P.ka * np.imag(np.vdot(np.asarray(pol, dtype=np.complex128), F))


def solve_sigma_ext(xyz, tri, k0, eps_r, khat, pol, mu_r=1.0, frame=0):
    P = galerkin.Problem(xyz, tri, k0, eps_r, mu_r, frame=frame)
    K = core.fill(xyz, tri, P.phys)
    Z = galerkin.assemble(P, *K)
    b = galerkin.planewave_rhs(P, np.asarray(khat)[None], np.asarray(pol)[None])[:, 0]
    x = np.linalg.solve(Z, b)
    return sigma_ext(P, x, khat, pol), x, Z, P


def richardson(f, a, h):
    """Central-difference derivative of f at a along the (complex) step h."""
    return (8.0 * (f(a + h) - f(a - h)) - (f(a + 2 * h) - f(a - 2 * h))) / (12.0 * h)


def dsigma_deps(xyz, tri, k0, eps_r, khat, pol, h=1e-3, frame=0):
    """(d sigma / d Re eps_r, d sigma / d Im eps_r) by differences."""
    eps_r = complex(eps_r)
    f_re = lambda t: solve_sigma_ext(xyz, tri, k0, eps_r + t, khat, pol, frame=frame)[0]
    f_im = lambda t: solve_sigma_ext(xyz, tri, k0, eps_r + 1j * t, khat, pol, frame=frame)[0]
    return richardson(f_re, 0.0, h), richardson(f_im, 0.0, h)


def dK_deps(xyz, tri, k0, eps_r, h=1e-3, mu_r=1.0, frame=0):
    """dK1, dK2eps, dK2mu / d eps_r (holomorphic) by differences of the fill."""
    def K(e):
        return np.stack(core.fill(xyz, tri, core.phys_vector(k0, e, mu_r, frame=frame)))
    return richardson(K, complex(eps_r), h)


def dsigma_ddirs(xyz, tri, k0, eps_r, khat, pol, dirs, h=1e-4, frame=0):
    """d sigma / dt for the node displacement x -> x + t dirs ([n_nodes, 3])."""
    f = lambda t: solve_sigma_ext(xyz + t * dirs, tri, k0, eps_r, khat, pol, frame=frame)[0]
    return richardson(f, 0.0, h)


def dsigma_dnormal(xyz, tri, k0, eps_r, khat, pol, weights, h=1e-4, frame=0):
    """d sigma / dt for the displacement x_v -> x_v + t weights_v n_v of
    every node, n_v the nodal normals of the unperturbed mesh (held fixed),
    by differences of the whole discrete map.  One node: a unit weight."""
    n0, _, _ = core.nodal_frames(xyz, tri)
    dirs = np.asarray(weights, dtype=np.float64)[:, None] * n0
    f = lambda t: solve_sigma_ext(xyz + t * dirs, tri, k0, eps_r, khat, pol, frame=frame)[0]
    return richardson(f, 0.0, h)
