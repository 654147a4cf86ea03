"""ctypes bindings of the oracle's C core (``mbem_oracle.c``).

TEST INFRASTRUCTURE ONLY: only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The C core is built
with the system gcc on first use (or by ``build()``).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mbem_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

PT_STRIDE = 25  # x(3) J n(3) t1(3) t2(3) s1(3) s2(3) N(6)


def build(force: bool = True) -> str:
    """Compile the oracle's C core with gcc -O2 -fopenmp."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if (not os.path.exists(_LIB)
                or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build(force=True)
        L = C.CDLL(_LIB)
        P = C.c_void_p
        i64 = C.c_int64
        L.or_rule7.argtypes = [P, P, P]
        L.or_rule12.argtypes = [P, P, P]
        L.or_gauss_legendre01.argtypes = [C.c_int, P, P]
        L.or_nodal_frames.argtypes = [P, i64, P, i64, P]
        L.or_point_data.argtypes = [P, i64, P, i64, i64, P, P, P, P]
        L.or_kernel_scalars.argtypes = [P, C.c_int, i64, P, P]
        L.or_pair_block.argtypes = [P, i64, P, i64, P, C.c_int, C.c_int, i64, i64, P]
        L.or_ss_rule.argtypes = [C.c_int, C.c_int, P]
        L.or_ss_rule.restype = i64
        L.or_fill.argtypes = [P, i64, P, i64, P, C.c_int, C.c_int, P, P, P]
        L.or_entries.argtypes = [P, i64, P, i64, P, C.c_int, C.c_int, i64, P, P, P]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _mesh(xyz, tri6):
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    tri6 = np.ascontiguousarray(tri6, dtype=np.int64)
    return xyz, tri6


def phys_vector(k0, eps_r, mu_r=1.0, variant=0, frame=0):
    """variant 0: 7-point regular rule, Sauter-Schwab on the full kernels,
    16-term series; 1: the paper's own scheme (12-point rule, Sauter-Schwab
    on the singular parts, the remainder by the 12-point rule, series
    truncated after n = 6).
    frame 0: basis N_j(y) t_beta(y) on the interpolated Gram-Schmidt frame
    (Sec. 3.3, Sec. 4.1); 1: node-attached tangents N_j(y) P(y) t_beta,j."""
    eps_r, mu_r = complex(eps_r), complex(mu_r)
    if frame not in (0, 1):
        raise ValueError(frame)
    return np.array([k0, eps_r.real, eps_r.imag, mu_r.real, mu_r.imag, float(variant),
                     float(frame)])


def rule7():
    xi, eta, w = (np.zeros(7) for _ in range(3))
    lib().or_rule7(_p(xi), _p(eta), _p(w))
    return xi, eta, w


def rule12():
    """(xi, eta, w) of the 12-point degree-6 rule on the reference triangle."""
    xi, eta, w = np.zeros(12), np.zeros(12), np.zeros(12)
    lib().or_rule12(_p(xi), _p(eta), _p(w))
    return xi, eta, w


def gauss_legendre01(n):
    x, w = np.zeros(n), np.zeros(n)
    if lib().or_gauss_legendre01(n, _p(x), _p(w)) != 0:
        raise ValueError(n)
    return x, w


def nodal_frames(xyz, tri6):
    """(n, t1, t2) each [n_nodes, 3]."""
    xyz, tri6 = _mesh(xyz, tri6)
    out = np.zeros((xyz.shape[0], 9))
    lib().or_nodal_frames(_p(xyz), xyz.shape[0], _p(tri6), tri6.shape[0], _p(out))
    return out[:, 0:3], out[:, 3:6], out[:, 6:9]


def point_data(xyz, tri6, elem, xi, eta):
    """Point data rows [npt, 25]: x J n t1 t2 s1 s2 N(6)."""
    xyz, tri6 = _mesh(xyz, tri6)
    elem = np.ascontiguousarray(elem, dtype=np.int64)
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    eta = np.ascontiguousarray(eta, dtype=np.float64)
    out = np.zeros((elem.shape[0], PT_STRIDE))
    lib().or_point_data(_p(xyz), xyz.shape[0], _p(tri6), tri6.shape[0],
                        elem.shape[0], _p(elem), _p(xi), _p(eta), _p(out))
    return out


def kernel_scalars(phys, R, mode=0):
    """D0, df, dg, G_eps, G_mu at distances R (mode 0 hybrid, 1 closed, 2 series,
    3 singular parts, 4 remainders = kernel - singular part)."""
    R = np.ascontiguousarray(R, dtype=np.float64)
    out = np.zeros((R.shape[0], 10))
    lib().or_kernel_scalars(_p(np.asarray(phys, dtype=np.float64)), mode,
                            R.shape[0], _p(R), _p(out))
    v = out[:, 0::2] + 1j * out[:, 1::2]
    return [v[:, k] for k in range(5)]


def pair_block(xyz, tri6, phys, e, f, nss=4, mode=0):
    """[6,6,12] complex block of element pair (e test, f trial)."""
    xyz, tri6 = _mesh(xyz, tri6)
    out = np.zeros(6 * 6 * 12 * 2)
    lib().or_pair_block(_p(xyz), xyz.shape[0], _p(tri6), tri6.shape[0],
                        _p(np.asarray(phys, dtype=np.float64)), nss, mode,
                        int(e), int(f), _p(out))
    return (out[0::2] + 1j * out[1::2]).reshape(6, 6, 12)


def ss_rule(cls, n):
    """Sauter-Schwab points on Th x Th: rows (s1, t1, s2, t2, weight)."""
    npt = lib().or_ss_rule(cls, n, None)
    out = np.zeros((npt, 5))
    lib().or_ss_rule(cls, n, _p(out))
    return out


def fill(xyz, tri6, phys, nss=4, nthreads=0):
    """Dense K1, K2^eps, K2^mu, each (2 nn)^2 complex128, user node order."""
    xyz, tri6 = _mesh(xyz, tri6)
    n2 = 2 * xyz.shape[0]
    K = [np.zeros((n2, n2), dtype=np.complex128) for _ in range(3)]
    rc = lib().or_fill(_p(xyz), xyz.shape[0], _p(tri6), tri6.shape[0],
                       _p(np.asarray(phys, dtype=np.float64)), nss, nthreads,
                       _p(K[0]), _p(K[1]), _p(K[2]))
    if rc:
        raise RuntimeError(f"or_fill failed {rc}")
    return K


def entries(xyz, tri6, phys, inode, jnode, nss=4, nthreads=0):
    """[ns, 3, 2, 2] complex node-pair entries (op, alpha, beta)."""
    xyz, tri6 = _mesh(xyz, tri6)
    inode = np.ascontiguousarray(inode, dtype=np.int64)
    jnode = np.ascontiguousarray(jnode, dtype=np.int64)
    out = np.zeros(inode.shape[0] * 24)
    lib().or_entries(_p(xyz), xyz.shape[0], _p(tri6), tri6.shape[0],
                     _p(np.asarray(phys, dtype=np.float64)), nss, nthreads,
                     inode.shape[0], _p(inode), _p(jnode), _p(out))
    return (out[0::2] + 1j * out[1::2]).reshape(-1, 3, 2, 2)
