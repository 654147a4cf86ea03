"""Morton ordering, Morton block-Jacobi and GMRES of the oracle (numpy).

TEST INFRASTRUCTURE ONLY.  Follows Sec. 5 of the paper:
 * a double Morton (Z-order) permutation, nodes first, then elements by the
   centroid of their three vertices;
 * contiguous clusters of B indices of one current's Morton-ordered vector;
   each preconditioner block is the 2B x 2B restriction of the full 2 x 2
   operator (eq. precond_block);
 * GMRES right-preconditioned by blockdiag(A_m).
"""
from __future__ import annotations

import numpy as np

MORTON_BITS = 21


def _spread3(v):
    """Put bit b of v at bit 3b (v < 2^21)."""
    out = np.zeros_like(v, dtype=np.uint64)
    for b in range(MORTON_BITS):
        out |= ((v >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b)
    return out


def morton_keys(points, lo, ext):
    """63-bit Z-order keys: cube-normalise by the bounding box's largest side,
    quantise to 21 bits per axis, interleave x -> bit 3b, y -> 3b+1, z -> 3b+2."""
    q = np.floor((points - lo[None, :]) / ext * float(1 << MORTON_BITS))
    q = np.clip(q, 0, (1 << MORTON_BITS) - 1).astype(np.uint64)
    return _spread3(q[:, 0]) | (_spread3(q[:, 1]) << np.uint64(1)) | \
        (_spread3(q[:, 2]) << np.uint64(2))


def morton_order(xyz, tri6):
    """(node_order, tri_order): Morton position k -> original index.

    Stable sort of the keys, ties broken by original index.
    """
    lo = xyz.min(axis=0)
    ext = float((xyz.max(axis=0) - lo).max())
    kn = morton_keys(xyz, lo, ext)
    node_order = np.argsort(kn, kind="stable")
    v = xyz[tri6[:, :3]]
    cen = ((v[:, 0] + v[:, 1]) + v[:, 2]) / 3.0
    ke = morton_keys(cen, lo, ext)
    tri_order = np.argsort(ke, kind="stable")
    return node_order, tri_order


def permute_unknowns(node_order):
    """Index map p with x_morton = x_user[p] for the 4 n_nodes unknowns."""
    nn = node_order.shape[0]
    one = np.stack([2 * node_order, 2 * node_order + 1], axis=1).ravel()
    return np.concatenate([one, 2 * nn + one])


def mbj_blocks(n2, B):
    """Clusters I_m = [m B, min((m+1) B, n2)) of one current's vector."""
    return [np.arange(s, min(s + B, n2)) for s in range(0, n2, B)]


def mbj_matrices(Z, B):
    """Preconditioner blocks A_m (eq. precond_block) of a Morton-ordered Z."""
    n2 = Z.shape[0] // 2
    out = []
    for I in mbj_blocks(n2, B):
        idx = np.concatenate([I, n2 + I])
        out.append(Z[np.ix_(idx, idx)])
    return out


def mbj_apply(blocks, v, B):
    n2 = v.shape[0] // 2
    z = np.zeros_like(v)
    for A, I in zip(blocks, mbj_blocks(n2, B)):
        idx = np.concatenate([I, n2 + I])
        z[idx] = np.linalg.solve(A, v[idx])
    return z


def gmres(matvec, b, precond=None, tol=1e-10, maxit=1000):
    """Right-preconditioned GMRES, x0 = 0, classical Gram-Schmidt applied
    twice, stop when the Arnoldi residual estimate reaches tol * |b|.

    Returns (x, iterations, residual history relative to |b|).
    """
    if precond is None:
        precond = lambda v: v  # noqa: E731
    n = b.shape[0]
    beta = np.linalg.norm(b)
    V = np.zeros((maxit + 1, n), dtype=np.complex128)
    H = np.zeros((maxit + 1, maxit), dtype=np.complex128)
    V[0] = b / beta
    g = np.zeros(maxit + 1, dtype=np.complex128)
    g[0] = beta
    cs = np.zeros(maxit, dtype=np.complex128)
    sn = np.zeros(maxit, dtype=np.complex128)
    hist = [1.0]
    k = 0
    for k in range(maxit):
        w = matvec(precond(V[k]))
        h = V[:k + 1].conj() @ w
        w = w - V[:k + 1].T @ h
        h2 = V[:k + 1].conj() @ w
        w = w - V[:k + 1].T @ h2
        h = h + h2
        hn = np.linalg.norm(w)
        H[:k + 1, k] = h
        H[k + 1, k] = hn
        if hn > 0:
            V[k + 1] = w / hn
        for i in range(k):
            t = cs[i] * H[i, k] + sn[i] * H[i + 1, k]
            H[i + 1, k] = -np.conj(sn[i]) * H[i, k] + cs[i] * H[i + 1, k]
            H[i, k] = t
        a, bb = H[k, k], H[k + 1, k]
        r = np.hypot(abs(a), abs(bb))
        cs[k] = abs(a) / r if r > 0 else 1.0
        sn[k] = (a / abs(a)) * np.conj(bb) / r if abs(a) > 0 else 1.0
        H[k, k] = cs[k] * a + sn[k] * bb
        H[k + 1, k] = 0.0
        g[k + 1] = -np.conj(sn[k]) * g[k]
        g[k] = cs[k] * g[k]
        hist.append(abs(g[k + 1]) / beta)
        if hist[-1] <= tol:
            k += 1
            break
    else:
        k = maxit
    y = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
    x = precond(V[:k].T @ y)
    return x, k, np.array(hist)


def cgemm_nt(A, B, conj_a=False):
    """C[b][m] = sum_k op(A[m][k]) B[b][k], op = conj when conj_a: the
    product of a block of row vectors B with a stored matrix A, written
    with the library matmul in complex128."""
    A = np.asarray(A, dtype=np.complex128)
    B = np.asarray(B, dtype=np.complex128)
    return B @ (A.conj() if conj_a else A).T


def solve_columns(Z, B):
    """X[c] with Z X[c] = B[c] for every row c of B (dense LU)."""
    return np.linalg.solve(np.asarray(Z, dtype=np.complex128),
                           np.asarray(B, dtype=np.complex128).T).T
