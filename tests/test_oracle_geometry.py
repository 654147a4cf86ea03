"""Pins of the oracle's P2 geometry, nodal normals and frames."""
import numpy as np
import pytest

from oracle import core, galerkin
from workloads import icosphere_p2


def _qp(xyz, tri):
    P = galerkin.Problem(xyz, tri, 1.0, 2.0)
    return P, P.qp()


@pytest.mark.parametrize("F", [80, 320, 1280])
def test_area_volume_converge_to_sphere(F):
    """P2 area -> 4 pi and enclosed volume int x.n/3 -> 4 pi/3."""
    xyz, tri = icosphere_p2(F)
    P, (elem, w, rows) = _qp(xyz, tri)
    WJ = w * rows[:, 3]
    area = WJ.sum()
    vol = np.sum(WJ * np.einsum("qd,qd->q", rows[:, 0:3], rows[:, 4:7])) / 3
    tol = {80: 5e-3, 320: 4e-4, 1280: 3e-5}[F]
    assert abs(area - 4 * np.pi) / (4 * np.pi) < tol
    assert abs(vol - 4 * np.pi / 3) / (4 * np.pi / 3) < tol


def test_area_convergence_rate():
    errs = []
    for F in (80, 320, 1280):
        xyz, tri = icosphere_p2(F)
        _, (elem, w, rows) = _qp(xyz, tri)
        errs.append(abs((w * rows[:, 3]).sum() - 4 * np.pi))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 3.5), rates   # P2 surface area error is O(h^4)


def test_mass_matrix_identities(sphere80):
    xyz, tri = sphere80
    P, (elem, w, rows) = _qp(xyz, tri)
    M = galerkin.mass_matrix(P).toarray()
    area = (w * rows[:, 3]).sum()
    assert np.abs(M - M.T).max() < 1e-16
    assert abs(M.sum() - area) < 1e-13
    assert np.linalg.eigvalsh(M).min() > 0
    # row sums = int N_i, and sum_i N_i = 1
    intN = np.zeros(P.nn)
    for k in range(6):
        np.add.at(intN, tri[elem, k], w * rows[:, 3] * rows[:, 19 + k])
    assert np.abs(M.sum(axis=1) - intN).max() < 1e-15
    assert np.abs(rows[:, 19:25].sum(axis=1) - 1).max() < 1e-15


def test_icosahedral_symmetry_normals(sphere80):
    """On the once-subdivided icosahedron the 12 original vertices lie on
    5-fold axes and the 30 original-edge midpoints on 2-fold axes of the
    mesh's symmetry group, so the metric-weighted normal must be radial there
    exactly (up to rounding)."""
    xyz, tri = sphere80
    n, t1, t2 = core.nodal_frames(xyz, tri)
    radial = xyz / np.linalg.norm(xyz, axis=1, keepdims=True)
    # vertices 0..11 are the icosahedron's, 12..41 the first-level midpoints
    err = np.linalg.norm(n[:42] - radial[:42], axis=1).max()
    assert err < 1e-14
    # elsewhere the normal is close to but not exactly radial
    assert np.linalg.norm(n[42:] - radial[42:], axis=1).max() > 1e-8


def test_triads_orthonormal_and_reference_axis(sphere80):
    xyz, tri = sphere80
    n, t1, t2 = core.nodal_frames(xyz, tri)
    for a in (n, t1, t2):
        assert np.abs(np.linalg.norm(a, axis=1) - 1).max() < 1e-15
    assert np.abs(np.einsum("vd,vd->v", n, t1)).max() < 1e-15
    assert np.abs(np.einsum("vd,vd->v", n, t2)).max() < 1e-15
    assert np.abs(np.einsum("vd,vd->v", np.cross(t1, t2), n) - 1).max() < 1e-15
    # t1 is orthogonal to the reference axis chosen by the 0.9 rule (Sec. 3.2)
    polar = np.abs(n[:, 2]) > 0.9
    assert np.abs(t1[polar, 0]).max() < 1e-15
    assert np.abs(t1[~polar, 2]).max() < 1e-15


def test_frames_tangent_at_quadrature_points(sphere80):
    """Exact tangency t_beta(y).n(y) = 0 (Sec. 3.3) and s_alpha = t_alpha x n."""
    xyz, tri = sphere80
    _, (elem, w, rows) = _qp(xyz, tri)
    n, t1, t2, s1, s2 = (rows[:, k:k + 3] for k in (4, 7, 10, 13, 16))
    assert np.abs(np.einsum("qd,qd->q", t1, n)).max() < 1e-15
    assert np.abs(np.einsum("qd,qd->q", t2, n)).max() < 1e-15
    assert np.abs(np.einsum("qd,qd->q", t1, t2)).max() < 1e-15
    assert np.abs(s1 + t2).max() < 1e-14 and np.abs(s2 - t1).max() < 1e-14
    # the P2 normal at a quadrature point is close to radial on the sphere
    radial = rows[:, 0:3] / np.linalg.norm(rows[:, 0:3], axis=1, keepdims=True)
    assert np.linalg.norm(n - radial, axis=1).max() < 2e-2


def _normal_error(F, axes):
    xyz, tri = icosphere_p2(F, axes)
    n = core.nodal_frames(xyz, tri)[0]
    a = np.asarray(axes)
    exact = xyz / a[None, :] ** 2
    exact /= np.linalg.norm(exact, axis=1, keepdims=True)
    return np.arccos(np.clip(np.einsum("vd,vd->v", n, exact), -1, 1)).max()


def test_normal_convergence_sphere_h3():
    """App. A: the metric-weighted normal converges O(h^3) on spheres."""
    e = [_normal_error(F, (1, 1, 1)) for F in (320, 1280, 5120)]
    rates = np.log2(np.array(e[:-1]) / np.array(e[1:]))
    assert np.all(rates > 2.6), rates


def test_normal_convergence_ellipsoid_h2():
    """App. A: O(h^2) on a general smooth surface."""
    e = [_normal_error(F, (1, 0.8, 0.6)) for F in (320, 1280, 5120)]
    rates = np.log2(np.array(e[:-1]) / np.array(e[1:]))
    assert np.all(rates > 1.7), rates
