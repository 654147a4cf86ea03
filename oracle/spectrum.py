"""Frequency / material sweep of the oracle (numpy).

TEST INFRASTRUCTURE ONLY.

A spectrum is the single-frequency path repeated on one mesh: at every
(k0, eps_r, mu_r) point the operator is filled, the system assembled and
solved densely, and the cross sections evaluated (Sec. 6.3, Benchmark II: the
LSPR spectrum of a silver spheroid, one solve per wavelength).  Nothing is
shared between points except the mesh.
"""
from __future__ import annotations

import numpy as np

from . import core, galerkin
from .galerkin import Problem


def spectrum(xyz, tri6, k0s, eps_rs, khat, pol, mu_rs=None, ntheta=None, variant=0, frame=0):
    """(C_ext, C_sca, C_abs)[npts, 3] for unit-amplitude incidence (khat [3],
    pol [3]) at every point; ntheta as galerkin.cross_sections (None: the
    default for each point's wavenumber)."""
    k0s = np.atleast_1d(np.asarray(k0s, dtype=np.float64))
    eps_rs = np.atleast_1d(np.asarray(eps_rs, dtype=np.complex128))
    mu_rs = np.ones_like(eps_rs) if mu_rs is None else np.atleast_1d(np.asarray(mu_rs, dtype=np.complex128))
    if not (k0s.shape == eps_rs.shape == mu_rs.shape):
        raise ValueError("k0s, eps_rs and mu_rs must have one entry per point")
    khat = np.asarray(khat, dtype=np.float64)
    pol = np.asarray(pol, dtype=np.complex128)
    out = np.zeros((k0s.shape[0], 3))
    for i, (k0, eps, mu) in enumerate(zip(k0s, eps_rs, mu_rs)):
        P = Problem(xyz, tri6, k0, eps, mu, variant=variant, frame=frame)
        K = core.fill(P.xyz, P.tri6, P.phys, nss=P.nss)
        Z = galerkin.assemble(P, K[0], K[1], K[2])
        x = np.linalg.solve(Z, galerkin.planewave_rhs(P, khat, pol))
        out[i] = galerkin.cross_sections(P, np.ravel(x), khat, pol, ntheta)
    return out

