"""Galerkin system, excitation and post-processing of the oracle (numpy).

TEST INFRASTRUCTURE ONLY.

Unknown layout: x = [c_j ; c_jm], each of length 2 n_nodes with index
2 * node + alpha in the caller's node order.  Units: eps_a = mu_a = 1,
eta_a = 1, omega = k_a = k0.

Tangential basis (``frame``): 0, the paper's printed construction, basis
vector N_j(y) t_beta(y) with t_beta(y) the interpolated Gram-Schmidt frame
(Sec. 3.3, Sec. 4.1); 1, node-attached tangents, N_j(y) P(y) t_beta,j with
t_beta,j the nodal triad's tangents (Sec. 3.2) and P(y) = I - n(y) n(y)^T.
The rotated test vector is (basis vector) x n in both.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import core


class Problem:
    """A mesh plus material: everything the oracle's formulas need."""

    def __init__(self, xyz, tri6, k0, eps_r, mu_r=1.0, nss=4, variant=0, frame=0):
        self.xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        self.tri6 = np.ascontiguousarray(tri6, dtype=np.int64)
        self.nn = self.xyz.shape[0]
        self.nt = self.tri6.shape[0]
        self.k0 = float(k0)
        self.eps_r = complex(eps_r)
        self.mu_r = complex(mu_r)
        self.nss = nss
        # variant selects the quadrature of the operator blocks (core.phys_vector);
        # mass matrix, right-hand side and far field keep the 7-point rule
        self.variant = variant
        self.frame = frame
        self.phys = core.phys_vector(k0, eps_r, mu_r, variant, frame)
        self.ka = self.k0
        ki = self.k0 * np.sqrt(self.eps_r * self.mu_r)
        self.ki = -ki if ki.imag < 0 else ki
        self.omega = self.k0
        self._qp = None
        self._basis = None

    # quadrature-point table on the 7-point rule -------------------------
    def qp(self):
        """(elem, w, rows[nt*7, 25]) at the 7 rule points of every element."""
        if self._qp is None:
            xi, eta, w = core.rule7()
            elem = np.repeat(np.arange(self.nt), 7)
            rows = core.point_data(self.xyz, self.tri6, elem,
                                   np.tile(xi, self.nt), np.tile(eta, self.nt))
            self._qp = (elem, np.tile(w, self.nt), rows)
        return self._qp

    def basis(self):
        """V[q, k, beta, 3]: the tangent vector that multiplies N_k in the
        basis function of local node k, component beta, at every 7-point rule
        point q (without the N_k factor)."""
        if self._basis is None:
            elem, w, rows = self.qp()
            V = np.zeros((elem.shape[0], 6, 2, 3))
            if self.frame == 0:
                V[:, :, 0, :] = rows[:, None, 7:10]
                V[:, :, 1, :] = rows[:, None, 10:13]
            else:
                n = rows[:, 4:7]
                _, t1n, t2n = core.nodal_frames(self.xyz, self.tri6)
                for b, tn in enumerate((t1n, t2n)):
                    t = tn[self.tri6[elem]]                              # q k 3
                    V[:, :, b, :] = t - np.sum(t * n[:, None, :], axis=2)[:, :, None] * n[:, None, :]
            self._basis = V
        return self._basis


def mass_matrix(P: Problem):
    """Scalar P2 Gram matrix M_ij = int N_i N_j (eq. mass_matrix), sparse."""
    elem, w, rows = P.qp()
    WJ = w * rows[:, 3]
    N = rows[:, 19:25]
    rr, cc, vv = [], [], []
    for k in range(6):
        for l in range(6):
            rr.append(P.tri6[elem, k])
            cc.append(P.tri6[elem, l])
            vv.append(WJ * N[:, k] * N[:, l])
    M = sp.coo_matrix((np.concatenate(vv), (np.concatenate(rr), np.concatenate(cc))),
                      shape=(P.nn, P.nn)).tocsr()
    return M


def mass_blocks(P: Problem):
    """Gram matrix of the vector basis, G[2i+a, 2j+b] = int N_i N_j V_ia . V_jb
    (eq. mass_matrix for the tangential functions), sparse 2nn x 2nn.  With
    the interpolated frame V_ia . V_jb = delta_ab and G = M (x) I_2."""
    if P.frame == 0:
        return sp.kron(mass_matrix(P), sp.identity(2), format="csr")
    elem, w, rows = P.qp()
    WJ = w * rows[:, 3]
    N = rows[:, 19:25]
    V = (N[:, :, None, None] * P.basis()).reshape(-1, 12, 3)
    dof = (2 * P.tri6[elem][:, :, None] + np.arange(2)[None, None, :]).reshape(-1, 12)
    G = np.einsum("q,qad,qbd->qab", WJ, V, V)
    r = np.repeat(dof[:, :, None], 12, axis=2).ravel()
    c = np.repeat(dof[:, None, :], 12, axis=1).ravel()
    return sp.coo_matrix((G.ravel(), (r, c)), shape=(2 * P.nn, 2 * P.nn)).tocsr()


def coefficients(P: Problem):
    """(i/omega, c_eps = (eps_i+eps_a)/2, c_mu = (mu_i+mu_a)/2) of eq. global_system."""
    return 1j / P.omega, (P.eps_r + 1.0) / 2.0, (P.mu_r + 1.0) / 2.0


def assemble(P: Problem, K1, K2e, K2m, M=None):
    """Dense Z of eq. global_system from the operator blocks and the mass:
    the scalar M (interpolated frame only) or, by default, mass_blocks."""
    if M is None:
        M2 = mass_blocks(P).toarray()
    elif M.shape[0] == P.nn:
        if P.frame != 0:
            raise ValueError("the scalar mass matrix only serves the interpolated frame")
        M2 = np.kron(M.toarray(), np.eye(2))
    else:
        M2 = M.toarray()
    iw, ce, cm = coefficients(P)
    return np.block([[iw * K1, ce * M2 + K2e], [cm * M2 + K2m, -iw * K1]])


def planewave_rhs(P: Problem, khat, pol):
    """b = [b_E ; b_H] for plane waves E = pol e^{i k_a khat.x} (eqs. rhs_E, rhs_H).

    khat[nrhs,3], pol[nrhs,3] -> b[4 n_nodes, nrhs] complex128.
    """
    khat = np.atleast_2d(np.asarray(khat, dtype=np.float64))
    pol = np.atleast_2d(np.asarray(pol, dtype=np.complex128))
    elem, w, rows = P.qp()
    WJ = w * rows[:, 3]
    x, n, N = rows[:, 0:3], rows[:, 4:7], rows[:, 19:25]
    S = np.cross(P.basis(), n[:, None, None, :])         # rotated test vectors
    nrhs = khat.shape[0]
    b = np.zeros((4 * P.nn, nrhs), dtype=np.complex128)
    for r in range(nrhs):
        ph = np.exp(1j * P.ka * (x @ khat[r]))
        E = ph[:, None] * pol[r][None, :]
        H = ph[:, None] * np.cross(khat[r], pol[r])[None, :]
        for a in range(2):
            for k in range(6):
                s = S[:, k, a, :]
                sE = np.einsum("qd,qd->q", s, E)
                sH = np.einsum("qd,qd->q", s, H)
                idx = 2 * P.tri6[elem, k] + a
                np.add.at(b[:, r], idx, -1.0 * WJ * N[:, k] * sE)
                np.add.at(b[:, r], 2 * P.nn + idx, 1.0 * WJ * N[:, k] * sH)
    return b


def surface_currents(P: Problem, x):
    """j and j_m at the 7 rule points of every element: [nt*7, 3] complex."""
    elem, w, rows = P.qp()
    N = rows[:, 19:25]
    V = P.basis()
    n2 = 2 * P.nn
    cj, cm = x[:n2], x[n2:]
    j = np.zeros((elem.shape[0], 3), dtype=np.complex128)
    jm = np.zeros_like(j)
    for k in range(6):
        node = P.tri6[elem, k]
        for b in range(2):
            t = V[:, k, b, :]
            j += (N[:, k] * cj[2 * node + b])[:, None] * t
            jm += (N[:, k] * cm[2 * node + b])[:, None] * t
    return j, jm


def far_field(P: Problem, x, rhat):
    """F(r) = (i k_a / 4 pi) r x int [eta_a j x r - j_m] e^{-i k_a r.y} dGamma_y.

    The radiation of the equivalent currents (Sec. 2.1 current definitions)
    into the exterior, normalised so that E_s ~ F e^{i k r} / r.
    rhat[ndir,3] -> F[ndir,3] complex.
    """
    rhat = np.atleast_2d(np.asarray(rhat, dtype=np.float64))
    elem, w, rows = P.qp()
    WJ = w * rows[:, 3]
    y = rows[:, 0:3]
    j, jm = surface_currents(P, x)
    F = np.zeros((rhat.shape[0], 3), dtype=np.complex128)
    for d in range(rhat.shape[0]):
        r = rhat[d]
        ph = WJ * np.exp(-1j * P.ka * (y @ r))
        integ = (ph[:, None] * (np.cross(j, r[None, :]) - jm)).sum(axis=0)
        F[d] = 1j * P.ka / (4 * np.pi) * np.cross(r, integ)
    return F


def sphere_quadrature(ntheta):
    """Gauss-Legendre in cos(theta) x trapezoid in phi (2 ntheta points)."""
    u, wu = np.polynomial.legendre.leggauss(ntheta)
    nphi = 2 * ntheta
    phi = 2 * np.pi * np.arange(nphi) / nphi
    th = np.arccos(u)
    T, Ph = np.meshgrid(th, phi, indexing="ij")
    W = (wu[:, None] * (2 * np.pi / nphi) * np.ones((1, nphi))).ravel()
    dirs = np.stack([np.sin(T) * np.cos(Ph), np.sin(T) * np.sin(Ph), np.cos(T)],
                    axis=-1).reshape(-1, 3)
    return dirs, W


def default_ntheta(P: Problem):
    amax = np.linalg.norm(P.xyz, axis=1).max()
    return int(np.ceil(2 * P.ka * amax)) + 20


def cross_sections(P: Problem, x, khat, pol, ntheta=None):
    """(C_ext, C_sca, C_abs) for unit-amplitude incidence.

    C_ext by the optical theorem (4 pi / k_a) Im(pol* . F(khat));
    C_sca = int |F|^2 dOmega on the sphere rule; C_abs = Re int n.(j_m x conj j).
    """
    khat = np.asarray(khat, dtype=np.float64)
    pol = np.asarray(pol, dtype=np.complex128)
    Ff = far_field(P, x, khat[None, :])[0]
    c_ext = 4 * np.pi / P.ka * np.imag(np.vdot(pol, Ff))
    if ntheta is None:
        ntheta = default_ntheta(P)
    dirs, W = sphere_quadrature(ntheta)
    F = far_field(P, x, dirs)
    c_sca = float(np.sum(W * np.sum(np.abs(F) ** 2, axis=1)))
    elem, w, rows = P.qp()
    WJ = w * rows[:, 3]
    n = rows[:, 4:7]
    j, jm = surface_currents(P, x)
    c_abs = float(np.real(np.sum(WJ * np.einsum("qd,qd->q", n, np.cross(jm, np.conj(j))))))
    return float(c_ext), c_sca, c_abs
