"""sigma_ext as a differentiable torch function of the permittivity and of
per-node normal displacements.

``SigmaExt.apply(eps, disp, ctx)`` with ``eps`` a real tensor [2] (Re, Im of
eps_r) and ``disp`` a real tensor [n_nodes] returns sigma_ext of the body
whose nodes are moved to x_v + disp_v n_v, n_v the nodal normals of the
undisplaced mesh (Sec. 3).  The forward pass runs fill, block-Jacobi setup,
GMRES and the far field in the HIP library; the backward pass runs the
library's adjoint (Z^T solve, dZ/deps_r fill and the reverse pass over the
geometry) and never differentiates through torch operations.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

from . import mbem


@dataclass
class SigmaExtProblem:
    """Fixed data of the map (eps_r, disp) -> sigma_ext."""
    xyz: np.ndarray                  # [n_nodes, 3] undisplaced nodes
    tri6: np.ndarray                 # [n_tris, 6]
    k0: float
    khat: np.ndarray                 # [3]
    pol: np.ndarray                  # [3] complex
    mu_r: complex = 1.0
    precision: int = mbem.MBEM_FP64
    frame: int = mbem.MBEM_FRAME_INTERPOLATED   # tangential basis (mbem.h)
    mbj_block: int = 100
    tol: float = 1e-12
    maxit: int = 600
    inner_tol: float = 1e-6
    normals: np.ndarray = field(default=None)   # filled on first use

    def nodal_normals(self):
        if self.normals is None:
            S = mbem.Solver(self.xyz, self.tri6, self.k0, 2.0)
            try:
                fr = S.nodal_frames()
            finally:
                S.close()
            self.normals = fr[:, 0:3].copy()
        return self.normals


def _forward(prob: SigmaExtProblem, eps: complex, disp: np.ndarray, want_grad: bool):
    xyz = prob.xyz + disp[:, None] * prob.nodal_normals()
    S = mbem.Solver(xyz, prob.tri6, prob.k0, eps, prob.mu_r, precision=prob.precision, frame=prob.frame)
    try:
        S.fill()
        S.precond_setup(prob.mbj_block)
        b = S.rhs(prob.khat[None], np.asarray(prob.pol)[None])
        x, st, code = S.solve(b, tol=prob.tol, maxit=prob.maxit, inner_tol=prob.inner_tol)
        if code != mbem.MBEM_OK:
            raise mbem.MbemError(code, "forward solve did not converge")
        # the nodes moved along the undisplaced normals, so the library
        # projects the position gradient on those, not on this mesh's normals
        res = S.grad_sigma_ext(x[0], prob.khat, prob.pol, tol=prob.tol, maxit=prob.maxit,
                               inner_tol=prob.inner_tol, shape=want_grad,
                               disp_dir=prob.nodal_normals() if want_grad else None)
        out = res[0]
        if not want_grad:
            return out[0], None, None
        return out[0], out[1:3].copy(), res[3].cpu().numpy()
    finally:
        S.close()


class SigmaExt(torch.autograd.Function):
    @staticmethod
    def forward(ctx, eps, disp, prob: SigmaExtProblem):
        e = eps.detach().cpu().numpy().astype(np.float64)
        d = disp.detach().cpu().numpy().astype(np.float64)
        want = eps.requires_grad or disp.requires_grad
        sig, geps, gdisp = _forward(prob, complex(e[0], e[1]), d, want)
        if want:
            ctx.save_for_backward(torch.as_tensor(geps, dtype=eps.dtype, device=eps.device),
                                  torch.as_tensor(gdisp, dtype=disp.dtype, device=disp.device))
        return torch.tensor(sig, dtype=torch.float64, device=eps.device)

    @staticmethod
    def backward(ctx, gout):
        geps, gdisp = ctx.saved_tensors
        return gout * geps, gout * gdisp, None
