"""Thin Python binding of the mbem C ABI (include/mbem.h).

Argument marshalling only: every step of the method runs in the HIP
library.  torch provides device memory (tensor data pointers) and the
stream.  Module-level functions carry the C names; ``Solver`` bundles the
handles for convenience.  Importing this module without the built library
raises immediately -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmbem.so")

MBEM_OK, MBEM_EINVAL, MBEM_ENOMEM, MBEM_EDEVICE = 0, -1, -2, -3
MBEM_ENOCONV, MBEM_ESINGULAR, MBEM_EMESH = -4, -5, -6
MBEM_FP64, MBEM_MIXED = 0, 1
MBEM_QUAD_DEFAULT, MBEM_QUAD_PAPER = 0, 1
MBEM_FRAME_INTERPOLATED, MBEM_FRAME_NODAL = 0, 1

EXPORTED = [
    "mbem_ctx_create", "mbem_ctx_destroy", "mbem_mesh_create", "mbem_mesh_destroy",
    "mbem_mesh_permutation", "mbem_mesh_info", "mbem_morton_order", "mbem_fill",
    "mbem_op_destroy", "mbem_op_export_blocks", "mbem_op_export_dense", "mbem_matvec",
    "mbem_precond_setup", "mbem_precond_apply", "mbem_rhs_planewave", "mbem_solve",
    "mbem_farfield", "mbem_cross_sections", "mbem_last_error", "mbem_solve_block",
    "mbem_gemm_autotune", "mbem_cgemm", "mbem_solve_adjoint", "mbem_fill_deps",
    "mbem_farfield_functional", "mbem_grad_sigma_ext", "mbem_mesh_frames", "mbem_spectrum",
    "mbem_fill_compressed", "mbem_matvec_noalloc",
]
GEMM_CONFIGS = 6   # FP32 GEMM tile shapes known to the autotuner


class MbemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mbem error {code}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [("k0", C.c_double), ("eps_r_re", C.c_double), ("eps_r_im", C.c_double),
                ("mu_r_re", C.c_double), ("mu_r_im", C.c_double), ("ssq_order", C.c_int32),
                ("precision", C.c_int32), ("near_radius", C.c_double), ("quadrature", C.c_int32),
                ("frame", C.c_int32), ("near_store", C.c_int32)]


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxit", C.c_int32), ("max_refine", C.c_int32),
                ("inner_tol", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("outer_iters", C.c_int32), ("rel_resid", C.c_double),
                ("t_fill_ms", C.c_double), ("t_setup_ms", C.c_double), ("t_solve_ms", C.c_double),
                ("n_near_pairs", C.c_int64), ("t_geom_ms", C.c_double),
                ("t_regular_ms", C.c_double), ("t_near_ms", C.c_double), ("t_ssq_ms", C.c_double),
                ("t_mass_ms", C.c_double), ("t_matvec_ms", C.c_double), ("n_matvec", C.c_int32),
                ("n_regular_pairs", C.c_int64), ("t_adjoint_ms", C.c_double),
                ("t_deps_ms", C.c_double), ("t_shape_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class BlrOpts(C.Structure):
    _fields_ = [("cluster", C.c_int32), ("eta", C.c_double), ("eps", C.c_double), ("rmax", C.c_int32),
                ("keep_lowrank", C.c_int32), ("band", C.c_int32)]


class BlrStats(C.Structure):
    _fields_ = [("stored_bytes", C.c_int64), ("dense_bytes", C.c_int64), ("n_clusters", C.c_int32),
                ("n_tiles", C.c_int32), ("n_admissible", C.c_int32), ("n_lowrank", C.c_int32),
                ("max_rank", C.c_int32), ("mean_rank", C.c_double), ("t_fill_ms", C.c_double),
                ("t_aca_ms", C.c_double), ("t_total_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class BlockOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("inner_tol", C.c_double), ("maxit", C.c_int32),
                ("max_refine", C.c_int32), ("block", C.c_int32), ("gemm_config", C.c_int32)]


class BlockStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("sweeps", C.c_int32), ("block", C.c_int32),
                ("gemm_config", C.c_int32), ("rel_resid", C.c_double), ("t_solve_ms", C.c_double),
                ("t_gemm_ms", C.c_double), ("n_gemm", C.c_int32), ("shifted", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """Load libmbem.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run paper_2604_21181_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        P, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
        PP = C.POINTER(C.c_void_p)
        sig = {
            "mbem_ctx_create": ([C.c_int, P, PP], C.c_int),
            "mbem_ctx_destroy": ([P], None),
            "mbem_mesh_create": ([P, P, i64, P, i64, PP], C.c_int),
            "mbem_mesh_destroy": ([P], None),
            "mbem_mesh_permutation": ([P, P, P], C.c_int),
            "mbem_mesh_info": ([P, P], C.c_int),
            "mbem_mesh_frames": ([P, P, P], C.c_int),
            "mbem_morton_order": ([P, i64, P, i64, P, P], C.c_int),
            "mbem_fill": ([P, P, C.POINTER(Params), PP, C.POINTER(Stats)], C.c_int),
            "mbem_op_destroy": ([P], None),
            "mbem_op_export_blocks": ([P, P, P, P, P], C.c_int),
            "mbem_op_export_dense": ([P, P, P], C.c_int),
            "mbem_matvec": ([P, P, P, i32, P], C.c_int),
            "mbem_matvec_noalloc": ([P, P, P, i32, P], C.c_int),
            "mbem_precond_setup": ([P, P, i32, C.POINTER(Stats)], C.c_int),
            "mbem_precond_apply": ([P, P, P, P], C.c_int),
            "mbem_rhs_planewave": ([P, P, C.POINTER(Params), P, P, i32, P], C.c_int),
            "mbem_solve": ([P, P, P, i32, C.POINTER(SolveOpts), P, C.POINTER(Stats)], C.c_int),
            "mbem_farfield": ([P, P, C.POINTER(Params), P, i32, P, i64, P], C.c_int),
            "mbem_cross_sections": ([P, P, C.POINTER(Params), P, P, P, i32, P], C.c_int),
            "mbem_last_error": ([], C.c_char_p),
            "mbem_solve_block": ([P, P, P, i32, C.POINTER(BlockOpts), P, C.POINTER(BlockStats)],
                                 C.c_int),
            "mbem_gemm_autotune": ([P, P, i32, i32, P, P], C.c_int),
            "mbem_cgemm": ([P, i32, i32, i64, i64, i64, P, i64, P, i64, P, i64, i32], C.c_int),
            "mbem_solve_adjoint": ([P, P, P, i32, C.POINTER(SolveOpts), P, C.POINTER(Stats)], C.c_int),
            "mbem_fill_deps": ([P, P, C.POINTER(Params), PP, C.POINTER(Stats)], C.c_int),
            "mbem_farfield_functional": ([P, P, C.POINTER(Params), P, P, P], C.c_int),
            "mbem_grad_sigma_ext": ([P, P, P, C.POINTER(Params), P, P, P, P, C.POINTER(SolveOpts), P, P,
                                     P, P, C.POINTER(Stats)], C.c_int),
            "mbem_spectrum": ([P, P, C.POINTER(Params), i32, P, P, P, P, P, i32,
                               C.POINTER(SolveOpts), i32, P, P, C.POINTER(Stats)], C.c_int),
            "mbem_fill_compressed": ([P, P, C.POINTER(Params), C.POINTER(BlrOpts), PP, C.POINTER(Stats),
                                      C.POINTER(BlrStats)], C.c_int),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(code, allow=()):
    if code != MBEM_OK and code not in allow:
        raise MbemError(code, lib().mbem_last_error().decode())
    return code


def _np_ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _t_ptr(t):
    return C.c_void_p(t.data_ptr())


def _check_vec(t, n, device, dtype=None, name="vector"):
    """Reject, before any library call, a tensor the kernels would read or
    write out of bounds: it must be a contiguous complex128 (or `dtype`)
    tensor on the solver's device with exactly n elements."""
    import torch
    dtype = torch.complex128 if dtype is None else dtype
    if not isinstance(t, torch.Tensor):
        raise MbemError(MBEM_EINVAL, f"{name}: expected a torch tensor, got {type(t).__name__}")
    if t.dtype != dtype:
        raise MbemError(MBEM_EINVAL, f"{name}: dtype {t.dtype}, expected {dtype}")
    if t.numel() != n:
        raise MbemError(MBEM_EINVAL, f"{name}: {t.numel()} elements, expected {n}")
    if not t.is_contiguous():
        raise MbemError(MBEM_EINVAL, f"{name}: not contiguous")
    if t.device != device:
        raise MbemError(MBEM_EINVAL, f"{name}: on {t.device}, expected {device}")
    return t


# ---------------------------------------------------------------- C names --
def mbem_ctx_create(device=0, stream=None):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(device).cuda_stream
    h = C.c_void_p()
    _check(lib().mbem_ctx_create(device, C.c_void_p(stream), C.byref(h)))
    return h


def mbem_ctx_destroy(ctx):
    lib().mbem_ctx_destroy(ctx)


def mbem_mesh_create(ctx, xyz, tri6):
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    tri6 = np.ascontiguousarray(tri6, dtype=np.int64)
    h = C.c_void_p()
    _check(lib().mbem_mesh_create(ctx, _np_ptr(xyz), xyz.shape[0], _np_ptr(tri6), tri6.shape[0],
                                  C.byref(h)))
    return h


def mbem_mesh_destroy(mesh):
    lib().mbem_mesh_destroy(mesh)


def mbem_mesh_info(mesh):
    info = np.zeros(8, dtype=np.int64)
    _check(lib().mbem_mesh_info(mesh, _np_ptr(info)))
    return info


def mbem_mesh_permutation(mesh):
    n = mbem_mesh_info(mesh)
    no = np.zeros(n[0], dtype=np.int64)
    to = np.zeros(n[1], dtype=np.int64)
    _check(lib().mbem_mesh_permutation(mesh, _np_ptr(no), _np_ptr(to)))
    return no, to


def mbem_morton_order(xyz, tri6):
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    tri6 = np.ascontiguousarray(tri6, dtype=np.int64)
    no = np.zeros(xyz.shape[0], dtype=np.int64)
    to = np.zeros(tri6.shape[0], dtype=np.int64)
    _check(lib().mbem_morton_order(_np_ptr(xyz), xyz.shape[0], _np_ptr(tri6), tri6.shape[0],
                                   _np_ptr(no), _np_ptr(to)))
    return no, to


def make_params(k0, eps_r, mu_r=1.0, precision=MBEM_FP64, ssq_order=4, near_radius=0.0,
                quadrature=MBEM_QUAD_DEFAULT, frame=MBEM_FRAME_INTERPOLATED, near_store=False):
    e, m = complex(eps_r), complex(mu_r)
    return Params(k0, e.real, e.imag, m.real, m.imag, ssq_order, precision, near_radius, quadrature, frame,
                  1 if near_store else 0)


def mbem_fill(ctx, mesh, params):
    h = C.c_void_p()
    st = Stats()
    _check(lib().mbem_fill(ctx, mesh, C.byref(params), C.byref(h), C.byref(st)))
    return h, st


def mbem_fill_compressed(ctx, mesh, params, cluster=256, eta=2.0, eps=1e-6, rmax=128, keep_lowrank=False,
                         band=0):
    """Block low-rank operator; returns (op, Stats, BlrStats)."""
    op = C.c_void_p()
    st, bs = Stats(), BlrStats()
    o = BlrOpts(cluster, eta, eps, rmax, 1 if keep_lowrank else 0, band)
    _check(lib().mbem_fill_compressed(ctx, mesh, C.byref(params), C.byref(o), C.byref(op), C.byref(st),
                                      C.byref(bs)))
    return op, st, bs


def mbem_op_destroy(op):
    lib().mbem_op_destroy(op)


def mbem_op_export_blocks(ctx, op, K1=None, K2e=None, K2m=None):
    p = [_t_ptr(t) if t is not None else None for t in (K1, K2e, K2m)]
    _check(lib().mbem_op_export_blocks(ctx, op, *p))


def mbem_op_export_dense(ctx, op, Z):
    _check(lib().mbem_op_export_dense(ctx, op, _t_ptr(Z)))


def mbem_matvec(ctx, op, x, y, nrhs=1):
    _check(lib().mbem_matvec(ctx, op, _t_ptr(x), nrhs, _t_ptr(y)))


def mbem_matvec_noalloc(ctx, op, x, y, nrhs=1):
    """Enqueue y = Z x without any allocation (the caller synchronises)."""
    _check(lib().mbem_matvec_noalloc(ctx, op, _t_ptr(x), nrhs, _t_ptr(y)))


def mbem_precond_setup(ctx, op, block):
    st = Stats()
    _check(lib().mbem_precond_setup(ctx, op, block, C.byref(st)))
    return st


def mbem_precond_apply(ctx, op, v, z):
    _check(lib().mbem_precond_apply(ctx, op, _t_ptr(v), _t_ptr(z)))


def mbem_rhs_planewave(ctx, mesh, params, khat, pol, b):
    khat = np.ascontiguousarray(np.atleast_2d(khat), dtype=np.float64)
    pol = np.ascontiguousarray(np.atleast_2d(pol), dtype=np.complex128)
    _check(lib().mbem_rhs_planewave(ctx, mesh, C.byref(params), _np_ptr(khat), _np_ptr(pol),
                                    khat.shape[0], _t_ptr(b)))


def mbem_solve(ctx, op, b, x, nrhs, tol, maxit=500, max_refine=0, inner_tol=0.0):
    o = SolveOpts(tol, maxit, max_refine, inner_tol)
    st = Stats()
    code = _check(lib().mbem_solve(ctx, op, _t_ptr(b), nrhs, C.byref(o), _t_ptr(x), C.byref(st)),
                  allow=(MBEM_ENOCONV,))
    return code, st


def mbem_solve_block(ctx, op, b, x, nrhs, tol, inner_tol=0.0, maxit=0, max_refine=0, block=0,
                     gemm_config=-1):
    o = BlockOpts(tol, inner_tol, maxit, max_refine, block, gemm_config)
    st = BlockStats()
    code = _check(lib().mbem_solve_block(ctx, op, _t_ptr(b), nrhs, C.byref(o), _t_ptr(x),
                                         C.byref(st)), allow=(MBEM_ENOCONV,))
    return code, st


def mbem_gemm_autotune(ctx, op, nrhs, reps=3):
    ms = np.zeros(GEMM_CONFIGS, dtype=np.float32)
    best = np.zeros(1, dtype=np.int32)
    _check(lib().mbem_gemm_autotune(ctx, op, nrhs, reps, _np_ptr(ms), _np_ptr(best)))
    return int(best[0]), ms


def mbem_cgemm(ctx, dtype, conj_a, A, B, C_out, config=0):
    """C_out[b][m] = sum_k op(A[m][k]) B[b][k] for row-major device tensors."""
    M, K = A.shape
    Nb = B.shape[0]
    _check(lib().mbem_cgemm(ctx, dtype, int(conj_a), M, Nb, K, _t_ptr(A), A.stride(0), _t_ptr(B),
                            B.stride(0), _t_ptr(C_out), C_out.stride(0), config))


def mbem_solve_adjoint(ctx, op, g, lam, nrhs, tol, maxit=500, max_refine=0, inner_tol=0.0):
    o = SolveOpts(tol, maxit, max_refine, inner_tol)
    st = Stats()
    code = _check(lib().mbem_solve_adjoint(ctx, op, _t_ptr(g), nrhs, C.byref(o), _t_ptr(lam),
                                           C.byref(st)), allow=(MBEM_ENOCONV,))
    return code, st


def mbem_fill_deps(ctx, mesh, params):
    op = C.c_void_p()
    st = Stats()
    _check(lib().mbem_fill_deps(ctx, mesh, C.byref(params), C.byref(op), C.byref(st)))
    return op, st


def mbem_farfield_functional(ctx, mesh, params, rhat, e, g):
    rhat = np.ascontiguousarray(rhat, dtype=np.float64).ravel()
    e = np.ascontiguousarray(e, dtype=np.complex128).ravel()
    _check(lib().mbem_farfield_functional(ctx, mesh, C.byref(params), _np_ptr(rhat), _np_ptr(e),
                                          _t_ptr(g)))


def mbem_grad_sigma_ext(ctx, op, mesh, params, x, khat, pol, tol=1e-12, maxit=500, inner_tol=0.0,
                        lam=None, dnode=None, dx=None, disp_dir=None):
    """disp_dir: host [n_nodes, 3] directions in Morton order, or None (nodal normals)."""
    khat = np.ascontiguousarray(khat, dtype=np.float64).ravel()
    pol = np.ascontiguousarray(pol, dtype=np.complex128).ravel()
    if khat.shape != (3,) or pol.shape != (3,):
        raise ValueError("khat and pol are 3-vectors")
    if disp_dir is not None:
        disp_dir = np.ascontiguousarray(disp_dir, dtype=np.float64)
        if disp_dir.ndim != 2 or disp_dir.shape[1] != 3:
            raise ValueError("disp_dir is [n_nodes, 3]")
    o = SolveOpts(tol, maxit, 0, inner_tol)
    out = np.zeros(3)
    st = Stats()
    opt = lambda t: _t_ptr(t) if t is not None else None
    _check(lib().mbem_grad_sigma_ext(ctx, op, mesh, C.byref(params), _t_ptr(x), _np_ptr(khat),
                                     _np_ptr(pol), _np_ptr(disp_dir) if disp_dir is not None else None,
                                     C.byref(o), _np_ptr(out), opt(lam), opt(dnode), opt(dx), C.byref(st)))
    return out, st


def mbem_farfield(ctx, mesh, params, x, nrhs, rhat, F):
    _check(lib().mbem_farfield(ctx, mesh, C.byref(params), _t_ptr(x), nrhs, _t_ptr(rhat),
                               rhat.shape[0], _t_ptr(F)))


def mbem_cross_sections(ctx, mesh, params, x, khat, pol, ntheta=0):
    khat = np.ascontiguousarray(khat, dtype=np.float64)
    pol = np.ascontiguousarray(pol, dtype=np.complex128)
    out = np.zeros(3)
    _check(lib().mbem_cross_sections(ctx, mesh, C.byref(params), _t_ptr(x), _np_ptr(khat),
                                     _np_ptr(pol), ntheta, _np_ptr(out)))
    return out


def mbem_spectrum(ctx, mesh, params, k0, eps_r, khat, pol, mu_r=None, block=100, tol=1e-5,
                  maxit=500, max_refine=0, inner_tol=0.0, ntheta=0):
    """Cross sections over (k0, eps_r[, mu_r]) points.  Returns
    (sigma[npts, 3] = C_ext, C_sca, C_abs; iters[npts]; Stats, summed).
    A point that missed the tolerance does not raise: its iteration count
    and stats.rel_resid show it."""
    k0 = np.ascontiguousarray(np.atleast_1d(k0), dtype=np.float64)
    eps = np.ascontiguousarray(np.atleast_1d(eps_r), dtype=np.complex128)
    mu = None if mu_r is None else np.ascontiguousarray(np.atleast_1d(mu_r), dtype=np.complex128)
    if eps.shape != k0.shape or (mu is not None and mu.shape != k0.shape):
        raise ValueError("k0, eps_r and mu_r need one entry per point")
    khat = np.ascontiguousarray(khat, dtype=np.float64).ravel()
    pol = np.ascontiguousarray(pol, dtype=np.complex128).ravel()
    if khat.shape != (3,) or pol.shape != (3,):
        raise ValueError("khat and pol are 3-vectors")
    sigma = np.zeros((k0.shape[0], 3))
    iters = np.zeros(k0.shape[0], dtype=np.int32)
    o = SolveOpts(tol, maxit, max_refine, inner_tol)
    st = Stats()
    _check(lib().mbem_spectrum(ctx, mesh, C.byref(params), k0.shape[0], _np_ptr(k0), _np_ptr(eps),
                               _np_ptr(mu) if mu is not None else None, _np_ptr(khat), _np_ptr(pol),
                               block, C.byref(o), ntheta, _np_ptr(sigma), _np_ptr(iters),
                               C.byref(st)), allow=(MBEM_ENOCONV,))
    return sigma, iters, st


# ------------------------------------------------------------- convenience --
class Solver:
    """Mesh + operator handles on one device; vectors are torch tensors in
    Morton order (``to_morton`` / ``to_user`` map caller-ordered arrays)."""

    def __init__(self, xyz, tri6, k0, eps_r, mu_r=1.0, precision=MBEM_FP64, ssq_order=4,
                 device=0, near_radius=0.0, quadrature=MBEM_QUAD_DEFAULT, frame=MBEM_FRAME_INTERPOLATED,
                 near_store=False):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.ctx = mbem_ctx_create(device)
        self.mesh = mbem_mesh_create(self.ctx, xyz, tri6)
        info = mbem_mesh_info(self.mesh)
        self.nn, self.nt, self.N = int(info[0]), int(info[1]), int(info[2])
        self.n_singular = (int(info[3]), int(info[4]), int(info[5]))
        self.node_order, self.tri_order = mbem_mesh_permutation(self.mesh)
        self.params = make_params(k0, eps_r, mu_r, precision, ssq_order, near_radius, quadrature, frame,
                                  near_store)
        self.op = None
        self.fill_stats = None

    # index map: x_morton = x_user[perm]
    @property
    def perm(self):
        no = self.node_order
        one = np.stack([2 * no, 2 * no + 1], 1).ravel()
        return np.concatenate([one, 2 * self.nn + one])

    def fill(self):
        if self.op is not None:
            mbem_op_destroy(self.op)
        self.op, self.fill_stats = mbem_fill(self.ctx, self.mesh, self.params)
        return self.fill_stats

    def fill_compressed(self, **kw):
        """Replace the operator by a block low-rank one (see
        mbem_fill_compressed); returns its BlrStats."""
        if self.op is not None:
            mbem_op_destroy(self.op)
            self.op = None
        self.op, self.fill_stats, bs = mbem_fill_compressed(self.ctx, self.mesh, self.params, **kw)
        return bs

    def export_blocks(self):
        t = self.torch
        n2 = 2 * self.nn
        K = [t.empty((n2, n2), dtype=t.complex128, device=self.device) for _ in range(3)]
        mbem_op_export_blocks(self.ctx, self.op, *K)
        t.cuda.synchronize()
        return K

    def export_dense(self):
        t = self.torch
        Z = t.empty((self.N, self.N), dtype=t.complex128, device=self.device)
        mbem_op_export_dense(self.ctx, self.op, Z)
        t.cuda.synchronize()
        return Z

    def matvec(self, x):
        nrhs = 1 if x.dim() == 1 else x.shape[0]
        x = _check_vec(x.contiguous(), nrhs * self.N, self.device, name="x")
        y = self.torch.empty_like(x)
        mbem_matvec(self.ctx, self.op, x, y, nrhs)
        return y

    def precond_setup(self, block):
        return mbem_precond_setup(self.ctx, self.op, block)

    def precond_apply(self, v):
        v = _check_vec(v.contiguous(), self.N, self.device, name="v")
        z = self.torch.empty_like(v)
        mbem_precond_apply(self.ctx, self.op, v, z)
        self.torch.cuda.synchronize()
        return z

    def rhs(self, khat, pol):
        khat = np.atleast_2d(khat)
        b = self.torch.empty((khat.shape[0], self.N), dtype=self.torch.complex128, device=self.device)
        mbem_rhs_planewave(self.ctx, self.mesh, self.params, khat, pol, b)
        return b

    def solve(self, b, tol, maxit=500, max_refine=0, inner_tol=0.0):
        b = b if b.dim() == 2 else b[None]
        b = _check_vec(b.contiguous(), b.shape[0] * self.N, self.device, name="b")
        x = self.torch.empty_like(b)
        code, st = mbem_solve(self.ctx, self.op, b, x, b.shape[0], tol, maxit, max_refine, inner_tol)
        return x, st, code

    def solve_block(self, b, tol, **kw):
        """b [nrhs, N] complex128 device tensor -> (x, BlockStats, code)."""
        if b.dim() != 2:
            raise MbemError(MBEM_EINVAL, "b: expected [nrhs, N]")
        b = _check_vec(b.contiguous(), b.shape[0] * self.N, self.device, name="b")
        x = self.torch.empty_like(b)
        code, st = mbem_solve_block(self.ctx, self.op, b, x, b.shape[0], tol, **kw)
        return x, st, code

    def solve_adjoint(self, g, tol, maxit=500, max_refine=0, inner_tol=0.0):
        g = g if g.dim() == 2 else g[None]
        g = _check_vec(g.contiguous(), g.shape[0] * self.N, self.device, name="g")
        lam = self.torch.empty_like(g)
        code, st = mbem_solve_adjoint(self.ctx, self.op, g, lam, g.shape[0], tol, maxit, max_refine,
                                      inner_tol)
        return lam, st, code

    def deps_blocks(self):
        """dK1, dK2eps, dK2mu / d eps_r (complex128 device tensors)."""
        t = self.torch
        dop, _ = mbem_fill_deps(self.ctx, self.mesh, self.params)
        try:
            n2 = 2 * self.nn
            K = [t.empty((n2, n2), dtype=t.complex128, device=self.device) for _ in range(3)]
            mbem_op_export_blocks(self.ctx, dop, *K)
            t.cuda.synchronize()
        finally:
            mbem_op_destroy(dop)
        return K

    def nodal_frames(self):
        """[n_nodes, 9]: nodal normal, t1, t2 in the caller's node order."""
        out = np.zeros((self.nn, 9))
        _check(lib().mbem_mesh_frames(self.ctx, self.mesh, _np_ptr(out)))
        return out

    def farfield_functional(self, rhat, e):
        g = self.torch.empty(self.N, dtype=self.torch.complex128, device=self.device)
        mbem_farfield_functional(self.ctx, self.mesh, self.params, rhat, e, g)
        return g

    def grad_sigma_ext(self, x, khat, pol, tol=1e-12, maxit=500, inner_tol=0.0, shape=False,
                       disp_dir=None):
        """(sigma_ext, d/dRe eps_r, d/dIm eps_r), adjoint-solve stats, lambda and,
        with shape=True, d sigma/d(node displacement) [n_nodes] along disp_dir
        ([n_nodes, 3] in the caller's node order; None: the nodal normals) and
        d sigma/d(node coordinates) [n_nodes, 3], both in the caller's node order."""
        t = self.torch
        x = _check_vec(x.reshape(-1).contiguous(), self.N, self.device, name="x")
        if disp_dir is not None:
            disp_dir = np.asarray(disp_dir, dtype=np.float64)
            if disp_dir.shape != (self.nn, 3):
                raise MbemError(MBEM_EINVAL, f"disp_dir: shape {disp_dir.shape}, expected ({self.nn}, 3)")
            disp_dir = disp_dir[self.node_order]          # Morton order
        lam = t.empty(self.N, dtype=t.complex128, device=self.device)
        dnode = t.empty(self.nn, dtype=t.float64, device=self.device) if shape else None
        dx = t.empty((self.nn, 3), dtype=t.float64, device=self.device) if shape else None
        out, st = mbem_grad_sigma_ext(self.ctx, self.op, self.mesh, self.params, x, khat, pol, tol,
                                      maxit, inner_tol, lam, dnode, dx, disp_dir=disp_dir)
        if not shape:
            return out, st, lam
        inv = t.as_tensor(np.argsort(self.node_order), device=self.device)
        return out, st, lam, dnode[inv], dx[inv]

    def gemm_autotune(self, nrhs, reps=3):
        return mbem_gemm_autotune(self.ctx, self.op, nrhs, reps)

    def farfield(self, x, rhat):
        t = self.torch
        x = x if x.dim() == 2 else x[None]
        x = _check_vec(x.contiguous(), x.shape[0] * self.N, self.device, name="x")
        r = t.as_tensor(np.ascontiguousarray(rhat, dtype=np.float64), device=self.device)
        F = t.empty((x.shape[0], r.shape[0], 3), dtype=t.complex128, device=self.device)
        mbem_farfield(self.ctx, self.mesh, self.params, x.contiguous(), x.shape[0], r, F)
        return F

    def cross_sections(self, x, khat, pol, ntheta=0):
        x = _check_vec(x.reshape(-1).contiguous(), self.N, self.device, name="x")
        return mbem_cross_sections(self.ctx, self.mesh, self.params, x, khat, pol, ntheta)

    def spectrum(self, k0, eps_r, khat, pol, mu_r=None, block=100, tol=1e-5, **kw):
        """Sweep on this solver's mesh with its precision and quadrature (its
        own k0 and materials are not used); see mbem_spectrum."""
        return mbem_spectrum(self.ctx, self.mesh, self.params, k0, eps_r, khat, pol, mu_r, block,
                             tol, **kw)

    def close(self):
        if self.op is not None:
            mbem_op_destroy(self.op)
            self.op = None
        if self.mesh is not None:
            mbem_mesh_destroy(self.mesh)
            self.mesh = None
        if self.ctx is not None:
            mbem_ctx_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
