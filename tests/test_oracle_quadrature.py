"""Pins of the oracle's quadrature rules (closed-form monomial integrals)."""
from math import factorial

import numpy as np
import pytest

from oracle import core


def tri_monomial(p, q):
    """int over {xi,eta>=0, xi+eta<=1} of xi^p eta^q = p! q! / (p+q+2)!"""
    return factorial(p) * factorial(q) / factorial(p + q + 2)


def test_rule7_exact_degree5():
    xi, eta, w = core.rule7()
    for p in range(6):
        for q in range(6 - p):
            v = np.sum(w * xi ** p * eta ** q)
            assert abs(v - tri_monomial(p, q)) < 1e-15, (p, q)
    # and not exact at degree 6 (a wrong rule of higher degree would pass
    # trivially; this pins the stated rule)
    errs = [abs(np.sum(w * xi ** p * eta ** (6 - p)) - tri_monomial(p, 6 - p))
            for p in range(7)]
    assert max(errs) > 1e-8


@pytest.mark.parametrize("n", [1, 2, 4, 7, 12])
def test_gauss_legendre_exact(n):
    x, w = core.gauss_legendre01(n)
    assert np.all(np.diff(x) > 0) and x[0] > 0 and x[-1] < 1
    for d in range(2 * n):
        assert abs(np.sum(w * x ** d) - 1.0 / (d + 1)) < 2e-15, d
    if n <= 7:  # the degree-2n error term is below rounding for larger n
        assert abs(np.sum(w * x ** (2 * n)) - 1.0 / (2 * n + 1)) > 1e-12


def th_monomial(a, b):
    """int over Th = {0 <= t <= s <= 1} of s^a t^b = 1/((b+1)(a+b+2))"""
    return 1.0 / ((b + 1) * (a + b + 2))


@pytest.mark.parametrize("cls", [3, 2, 1])
@pytest.mark.parametrize("n,maxdeg", [(4, 4), (8, 6)])
def test_sauter_schwab_polynomial_exact(cls, n, maxdeg):
    """The Sauter-Schwab regions must tile Th x Th exactly: every monomial
    s1^a t1^b s2^c t2^d of total degree <= maxdeg integrates to the product
    of the two single-triangle integrals."""
    R = core.ss_rule(cls, n)
    assert R.shape[0] == {3: 6, 2: 5, 1: 2}[cls] * n ** 4
    s1, t1, s2, t2, w = R.T
    assert np.all(t1 <= s1 + 1e-15) and np.all(t2 <= s2 + 1e-15)
    assert np.all(t1 >= 0) and np.all(s1 <= 1) and np.all(t2 >= 0) and np.all(s2 <= 1)
    for a in range(maxdeg + 1):
        for b in range(maxdeg + 1 - a):
            for c in range(maxdeg + 1 - a - b):
                for d in range(maxdeg + 1 - a - b - c):
                    v = np.sum(w * s1 ** a * t1 ** b * s2 ** c * t2 ** d)
                    ex = th_monomial(a, b) * th_monomial(c, d)
                    assert abs(v - ex) < 1e-15, (a, b, c, d)


def _flat_map(P0, P1, P2, s, t):
    """Point of the flat triangle (P0, P1, P2) at Th coordinates (s, t):
    (s,t) -> (xi,eta) = (s - t, t) -> P0 + xi (P1 - P0) + eta (P2 - P0)."""
    xi, eta = s - t, t
    return P0 + xi[:, None] * (P1 - P0) + eta[:, None] * (P2 - P0)


def _ss_inv_r(cls, n, T1, T2):
    """int int 1/|x-y| over two flat triangles with the shared vertices
    listed first in the same order (T = (P0, P1, P2))."""
    s1, t1, s2, t2, w = core.ss_rule(cls, n).T
    x = _flat_map(*T1, s1, t1)
    y = _flat_map(*T2, s2, t2)
    A1 = np.linalg.norm(np.cross(T1[1] - T1[0], T1[2] - T1[0]))
    A2 = np.linalg.norm(np.cross(T2[1] - T2[0], T2[2] - T2[0]))
    return A1 * A2 * np.sum(w / np.linalg.norm(x - y, axis=1))


def test_sauter_schwab_subdivision_identity():
    """Split a flat triangle T into its 4 midpoint children.  For the 1/R
    kernel (homogeneous of degree -1 in 4 dimensions) each child's self
    integral is 1/8 of T's, so
        I_coinc(T) / 2 = sum of the 6 ordered edge-adjacent child pairs
                         + the 6 ordered vertex-adjacent child pairs.
    This ties the three singular classes to each other on a singular kernel."""
    A = np.array([0.0, 0.0, 0.0])
    B = np.array([1.3, 0.1, 0.0])
    Cc = np.array([0.4, 0.9, 0.2])
    mab, mbc, mca = (A + B) / 2, (B + Cc) / 2, (Cc + A) / 2
    n = 12
    I_T = _ss_inv_r(3, n, (A, B, Cc), (A, B, Cc))
    corners = [(A, mab, mca), (B, mbc, mab), (Cc, mca, mbc)]
    center = (mab, mbc, mca)
    total = 0.0
    # centre child shares one edge with each corner child
    for (P, Q, R) in corners:
        # corner (P, Q, R) shares edge (Q, R) with the centre
        cen_third = [v for v in center if not (np.allclose(v, Q) or np.allclose(v, R))][0]
        total += _ss_inv_r(2, n, (Q, R, P), (Q, R, cen_third))
        total += _ss_inv_r(2, n, (Q, R, cen_third), (Q, R, P))
    # corner children share one vertex pairwise
    for i in range(3):
        for j in range(3):
            if i == j:
                continue
            Ti, Tj = corners[i], corners[j]
            shared = [v for v in Ti if any(np.allclose(v, u) for u in Tj)][0]
            oi = [v for v in Ti if not np.allclose(v, shared)]
            oj = [v for v in Tj if not np.allclose(v, shared)]
            total += _ss_inv_r(1, n, (shared, *oi), (shared, *oj))
    assert abs(total - I_T / 2) / I_T < 1e-11


def test_sauter_schwab_self_integral_converges():
    """Cauchy convergence of the coincident rule on 1/R (exponential)."""
    T = (np.array([0.0, 0, 0]), np.array([1.0, 0, 0]), np.array([0.3, 0.8, 0]))
    v = [_ss_inv_r(3, n, T, T) for n in (4, 8, 16)]
    assert abs(v[1] - v[2]) / v[2] < 1e-9
    assert abs(v[0] - v[2]) / v[2] < 1e-4
