"""The oracle's version of the paper's own quadrature scheme (variant 1):
12-point regular rule, Sauter-Schwab on the singular kernels kappa^s only,
the remainder kappa - kappa^s by the 12-point rule, Taylor series truncated
after n = 6.

Pins:
  * the 12-point rule integrates every monomial of degree <= 6 exactly on
    the reference triangle (and not every one of degree 7), and its seven
    parameters solve the moment equations of the S3-invariant polynomials
    (Newton from the printed 15-digit values reproduces the table);
  * the truncated H_diff equals the paper's five-term expansion
    (eq. H_diff_truncated) written out from its printed coefficients;
  * the singular parts are the paper's kappa_1^s / (grad Phi)^s
    (eq. kappa_S and the expansion of grad phi of Sec. 4.2); singular part +
    remainder = kernel at every distance; the remainder is continuous at
    R = 0, where its values are the R^0 terms of the paper's expansions;
  * singular-pair blocks of the variant converge to those of the default
    scheme (Sauter-Schwab on the full kernel at a high order) and regular
    blocks of the two rules agree to the quadrature error.
"""
from fractions import Fraction
from math import factorial

import numpy as np
import pytest

from oracle import core, galerkin
from workloads import icosphere_p2


# ------------------------------------------------------------ the rule --
def _tri_monomial(a, b):
    """int over {x, y >= 0, x + y <= 1} of x^a y^b."""
    return factorial(a) * factorial(b) / factorial(a + b + 2)


def test_rule12_exact_to_degree_6():
    xi, eta, w = core.rule12()
    assert np.all(w > 0) and np.all(xi > 0) and np.all(eta > 0) and np.all(xi + eta < 1)
    assert abs(w.sum() - 0.5) < 1e-15
    for a in range(7):
        for b in range(7 - a):
            assert abs(np.sum(w * xi ** a * eta ** b) - _tri_monomial(a, b)) < 2e-16, (a, b)
    err7 = max(abs(np.sum(w * xi ** a * eta ** (7 - a)) - _tri_monomial(a, 7 - a)) for a in range(8))
    assert err7 > 1e-8


def _moment_equations():
    def mono(a, b, c):
        return Fraction(2 * factorial(a) * factorial(b) * factorial(c), factorial(a + b + c + 2))

    def mul(p, q):
        r = {}
        for e1, c1 in p.items():
            for e2, c2 in q.items():
                e = tuple(x + y for x, y in zip(e1, e2))
                r[e] = r.get(e, 0) + c1 * c2
        return r
    E2 = {(1, 1, 0): 1, (0, 1, 1): 1, (1, 0, 1): 1}
    E3 = {(1, 1, 1): 1}
    conds = [(i, j) for i in range(4) for j in range(3) if 2 * i + 3 * j <= 6]
    exact = []
    for i, j in conds:
        p = {(0, 0, 0): 1}
        for _ in range(i):
            p = mul(p, E2)
        for _ in range(j):
            p = mul(p, E3)
        exact.append(float(sum(Fraction(c) * mono(*e) for e, c in p.items())))

    def points(u):
        a1, w1, a2, w2, b, c, w3 = u
        P, W = [], []
        for a, w in ((a1, w1), (a2, w2)):
            for k in range(3):
                l = [a, a, a]
                l[k] = 1 - 2 * a
                P.append(l)
                W.append(w)
        for perm in ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)):
            l = [0.0, 0.0, 0.0]
            for k, v in zip(perm, (b, c, 1 - b - c)):
                l[k] = v
            P.append(l)
            W.append(w3)
        return np.array(P), np.array(W)

    def F(u):
        P, W = points(u)
        e2 = P[:, 0] * P[:, 1] + P[:, 1] * P[:, 2] + P[:, 2] * P[:, 0]
        e3 = P[:, 0] * P[:, 1] * P[:, 2]
        return np.array([np.sum(W * e2 ** i * e3 ** j) for i, j in conds]) - np.array(exact)
    return F, points


def test_rule12_solves_the_moment_equations():
    """Newton on the seven invariant moment equations, started from the
    printed 15-digit parameters, lands on the oracle's table."""
    F, points = _moment_equations()
    u = np.array([0.063089014491502, 0.050844906370207, 0.249286745170910, 0.116786275726379,
                  0.053145049844817, 0.310352451033784, 0.082851075618374])
    for _ in range(4):
        J = np.zeros((7, 7))
        for k in range(7):
            d = np.zeros(7)
            d[k] = 1e-7
            J[:, k] = (F(u + d) - F(u - d)) / 2e-7
        u = u - np.linalg.solve(J, F(u))
    assert np.abs(F(u)).max() < 1e-15
    P, W = points(u)
    xi, eta, w = core.rule12()
    # same points (barycentric (1 - xi - eta, xi, eta)) in the same order, to
    # the conditioning of the moment system
    assert np.abs(P[:, 1] - xi).max() < 1e-13 and np.abs(P[:, 2] - eta).max() < 1e-13
    assert np.abs(0.5 * W - w).max() < 1e-14
    # and the table's own parameters solve the equations to rounding
    l0 = 1 - xi[6] - eta[6]                      # the (b, c, 1 - b - c) orbit, identity order
    tab = np.array([xi[0], 2 * w[0], xi[3], 2 * w[3], l0, xi[6], 2 * w[6]])
    assert np.abs(F(tab)).max() < 1e-15


# ------------------------------------------- kernels of the variant --
K0, EPS = 3.0, 4.0 + 0.3j


def _k():
    ka = K0
    ki = K0 * np.sqrt(EPS)
    return ka, (-ki if ki.imag < 0 else ki)


def test_truncated_hdiff_is_the_papers_five_terms():
    """H_diff = df Rh Rh^T - dg I of the variant's series (n <= 6) against
    the five printed terms of eq. H_diff_truncated."""
    ph = core.phys_vector(K0, EPS, 1.0, variant=1)
    R = np.array([1e-3, 0.01, 0.05, 0.1])
    D0, df, dg, Ge, Gm = core.kernel_scalars(ph, R, mode=2)
    ka, ki = _k()
    A = (ka ** 2 - ki ** 2) / (8 * np.pi * R)          # (Rh Rh - I)
    B = -1j * (ka ** 3 - ki ** 3) / (12 * np.pi)        # I
    C = (ka ** 4 - ki ** 4) / (32 * np.pi) * R          # (Rh Rh + I)
    D = 1j * (ka ** 5 - ki ** 5) / (120 * np.pi) * R ** 2  # (2 Rh Rh + I)
    E = -(ka ** 6 - ki ** 6) / (576 * np.pi) * R ** 3      # (3 Rh Rh + I)
    rr = A + C + 2 * D + 3 * E                          # coefficient of Rh Rh
    ii = -A + B + C + D + E                             # coefficient of I
    assert np.allclose(df, rr, rtol=1e-13, atol=0)
    assert np.allclose(-dg, ii, rtol=1e-13, atol=0)


def test_singular_parts_and_remainders():
    ka, ki = _k()
    ph = core.phys_vector(K0, EPS, 1.0, variant=1)
    R = np.array([1e-6, 1e-3, 0.03, 0.08, 0.2, 0.5, 1.3])   # both sides of max|k| R = 1/2
    full = core.kernel_scalars(ph, R, mode=0)
    sing = core.kernel_scalars(ph, R, mode=3)
    rem = core.kernel_scalars(ph, R, mode=4)
    # the paper's singular kernels: kappa_1^s carries (k_a^2 - k_i^2)/(8 pi R) on
    # [s.t + (s.Rh)(Rh.t)], i.e. D0^s - dg^s and df^s both equal that factor
    # while D0^s = 2 x it; (grad Phi_eps)^s = -(eps_a - eps_i)/(4 pi R^2) Rh
    f = (ka ** 2 - ki ** 2) / (8 * np.pi * R)
    assert np.allclose(sing[0], 2 * f, rtol=1e-15) and np.allclose(sing[1], f, rtol=1e-15)
    assert np.allclose(sing[2], f, rtol=1e-15)
    assert np.allclose(sing[3], -(1.0 - EPS) / (4 * np.pi * R ** 2), rtol=1e-15)
    assert np.allclose(sing[4], np.zeros_like(R), atol=0)          # mu_a = mu_i = 1
    # singular part + remainder = kernel (the full kernel uses the same
    # truncated series below max|k| R = 1/2)
    for k in range(5):
        scale = np.abs(full[k]) + np.abs(sing[k])
        assert np.all(np.abs(sing[k] + rem[k] - full[k]) <= 1e-12 * scale + 1e-300), k
    # R = 0: the R^0 terms of the paper's expansions
    z = core.kernel_scalars(ph, np.array([0.0]), mode=4)
    assert abs(z[0][0] - 1j * (ka ** 3 - ki ** 3) / (4 * np.pi)) < 1e-14 * abs(ka ** 3 - ki ** 3)
    assert abs(z[1][0]) == 0.0
    assert abs(z[2][0] - 1j * (ka ** 3 - ki ** 3) / (12 * np.pi)) < 1e-14 * abs(ka ** 3 - ki ** 3)
    # grad phi_chi = (1/4 pi)(-1/R^2 - k^2/2 + O(R)) Rh (Sec. 4.2), chi-weighted
    g0 = -(1.0 * ka ** 2 - EPS * ki ** 2) / (8 * np.pi)
    assert abs(z[3][0] - g0) < 1e-14 * abs(g0)
    # continuity at R = 0
    small = core.kernel_scalars(ph, np.array([1e-9]), mode=4)
    for k in range(5):
        assert abs(small[k][0] - z[k][0]) < 1e-7 * (abs(z[k][0]) + 1), k


# ------------------------------------------------------ blocks --------
def _pairs(tri):
    """one coincident, one common-edge, one common-vertex and one regular pair."""
    e = 0
    te = set(tri[e, :3])
    out = {3: (e, e)}
    for f in range(tri.shape[0]):
        n = len(te & set(tri[f, :3]))
        if n in (1, 2) and n not in out:
            out[n] = (e, f)
        if n == 0 and 0 not in out:
            out[0] = (e, f)
    return out


@pytest.mark.parametrize("cls", [3, 2, 1])
def test_variant_singular_blocks_match_full_kernel_ssq(cls):
    """Variant (Sauter-Schwab on kappa^s + 12-point rule on the remainder)
    against Sauter-Schwab on the full kernel at order 10, mu_r = 2 so that
    all three operators have a singular part.  The remainder is bounded but
    not smooth at coincidence (R^1 terms, the direction of grad Phi), and
    it is proportional to k^2, so the difference falls as k^2: a wrong
    singular part would leave a k-independent difference instead."""
    xyz, tri = icosphere_p2(80)
    e, f = _pairs(tri)[cls]
    err = {}
    for k0 in (1.0, 0.3):
        ref = core.pair_block(xyz, tri, core.phys_vector(k0, 4.0, 2.0), e, f, nss=10)
        var = core.pair_block(xyz, tri, core.phys_vector(k0, 4.0, 2.0, variant=1), e, f, nss=10)
        err[k0] = [np.abs(var[:, :, 4 * o:4 * o + 4] - ref[:, :, 4 * o:4 * o + 4]).max()
                   / np.abs(ref[:, :, 4 * o:4 * o + 4]).max() for o in range(3)]
    assert max(err[0.3]) < 2e-3, err
    if cls > 1:        # vertex pairs are already at the level of the rules' own error
        for o in range(3):
            assert err[1.0][o] > 5 * err[0.3][o], (o, err)
    # the singular part converges under the Sauter-Schwab order
    v4 = core.pair_block(xyz, tri, core.phys_vector(1.0, 4.0, 2.0, variant=1), e, f, nss=4)
    v8 = core.pair_block(xyz, tri, core.phys_vector(1.0, 4.0, 2.0, variant=1), e, f, nss=8)
    assert np.abs(v4 - v8).max() / np.abs(v8).max() < 1e-3


def test_variant_regular_block_close_to_the_7_point_rule():
    """Regular pairs: the degree-5 and degree-6 rules differ by the 7-point
    rule's quadrature error, which shrinks as the kernels vary less over an
    element (lower k) and is largest for neighbouring triangles."""
    xyz, tri = icosphere_p2(80)
    c = xyz[tri[:, :3]].mean(axis=1)
    e = 0
    far = int(np.argmax(np.linalg.norm(c - c[e], axis=1)))
    near = _pairs(tri)[0][1]
    d = {}
    for k0 in (3.0, 1.0):
        for f in (far, near):
            b7 = core.pair_block(xyz, tri, core.phys_vector(k0, EPS), e, f)
            b12 = core.pair_block(xyz, tri, core.phys_vector(k0, EPS, variant=1), e, f)
            d[k0, f] = np.abs(b12 - b7).max() / np.abs(b12).max()
    for f in (far, near):
        assert 0 < d[1.0, f] < d[3.0, f] < 1e-2, d
    assert d[1.0, far] < d[1.0, near], d


def test_variant_operator_far_field_close_to_default():
    """Whole operator: the far fields of the two schemes differ by their
    quadrature errors, which shrink under refinement (80 -> 320 triangles);
    both stay at the level of the discretisation error against Mie."""
    from oracle import mie, solve_dense
    kh = np.array([[0.0, 0.0, 1.0]])
    pol = np.array([[1.0, 0.0, 0.0]], dtype=np.complex128)
    r = np.array([[np.sin(t), 0.0, np.cos(t)] for t in np.linspace(0, np.pi, 19)])
    Fm = mie.far_field(1.0, 1.0, 4.0, r)
    diff = {}
    for nt in (80, 320):
        xyz, tri = icosphere_p2(nt)
        F = []
        for v in (0, 1):
            P = galerkin.Problem(xyz, tri, 1.0, 4.0, variant=v)
            x = solve_dense(P, kh, pol)[0][:, 0]
            F.append(galerkin.far_field(P, x, r))
            assert np.linalg.norm(F[-1] - Fm) / np.linalg.norm(Fm) < 3e-2
        diff[nt] = np.linalg.norm(F[1] - F[0]) / np.linalg.norm(F[0])
    assert diff[320] < diff[80] < 3e-3, diff
