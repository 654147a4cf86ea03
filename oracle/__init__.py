"""Plain FP64 CPU oracle of the nodal P2 Mueller BEM hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the HIP library: geometry, quadrature, kernels, Sauter-Schwab maps,
Morton ordering and the solver are all written again here, in the most
direct form, from the paper (arXiv 2604.21181):

  core.py      C core (FP64): P2 geometry, nodal frames, kernels, pair
               quadrature (7-point rule and Sauter-Schwab), dense fill,
               single node-pair entries
  galerkin.py  tangential basis (interpolated frame or node-attached
               tangents), mass matrix, system assembly, plane-wave
               excitation, far field and cross sections
  solver.py    Morton order, Morton block-Jacobi, GMRES
  mie.py       Mie series (spheres)
  spectrum.py  sweeps over wavenumber and material on one mesh
  blr.py       block low-rank compression of the operator blocks (ACA)

Parity status of every function is listed in the design notes; everything
here is pinned by the CPU test-suite (quadrature exactness, closed forms,
symmetry, zero contrast, Mie).
"""
from __future__ import annotations

import numpy as np

from . import blr, core, galerkin, mie, solver, spectrum
from .galerkin import Problem

__all__ = ["blr", "core", "galerkin", "mie", "solver", "spectrum", "Problem", "solve_dense"]


def solve_dense(P: Problem, khat, pol, K=None):
    """Fill, assemble and solve by dense LU.  Returns (x[4nn, nrhs], K, G)
    with G the Gram matrix of the tangential basis (galerkin.mass_blocks)."""
    if K is None:
        K = core.fill(P.xyz, P.tri6, P.phys, nss=P.nss)
    M = galerkin.mass_blocks(P)
    Z = galerkin.assemble(P, K[0], K[1], K[2], M)
    b = galerkin.planewave_rhs(P, khat, pol)
    x = np.linalg.solve(Z, b)
    return x, K, M
