"""Block low-rank (BLR) compression of the operator blocks (numpy).

TEST INFRASTRUCTURE ONLY.

The paper leaves compressed far-field interactions to future work (Sec. 7, Conclusion,
FMM for problems beyond dense memory).  The compressed operator checked
here is defined as follows, on the Morton-ordered nodes of Sec. 5:

  * clusters: the leaves of the octree of the nodes' Morton keys (63 bits,
    Sec. 5): the nodes sharing the top 3 l key bits form a cell of level l,
    a contiguous run of the Morton order; a cell with more than L nodes is
    split into its children (the runs sharing 3 (l + 1) bits), down to level
    21, where a run still longer than L is cut into pieces of L.  Cluster c
    owns rows / columns 2 i + alpha of every operator block for its nodes i;
  * support box of a cluster: the axis-aligned bounding box of the six nodes
    of every element that has a node in the cluster (it holds the support of
    every basis function of the cluster);
  * a cluster pair (t, s) is admissible when t != s, the boxes are apart
    (dist > 0) and max(diam_t, diam_s) <= eta * dist (diam: box diagonal);
  * admissible tiles of K1, K2^eps, K2^mu are replaced by the rank-k
    approximation of adaptive cross approximation with partial pivoting
    (Bebendorf, Numer. Math. 86 (2000); stopping rule |u_k| |v_k| <=
    eps |S_k|_F), tiles whose approximation does not converge within rmax
    terms or saves no memory stay dense, and every other tile is dense;
  * the mass matrix (local) is untouched.
"""
from __future__ import annotations

import numpy as np


def node_keys(xyz_m):
    """Morton keys of the Morton-ordered nodes (non-decreasing)."""
    from . import solver
    lo = xyz_m.min(axis=0)
    ext = float((xyz_m.max(axis=0) - lo).max())
    return solver.morton_keys(xyz_m, lo, ext)


def clusters(keys, L):
    """[(first, last + 1)] node ranges of the octree leaves (see above)."""
    out = []

    def split(a, b, lev):
        if b - a <= L:
            out.append((a, b))
            return
        if lev == 21:
            out.extend((s, min(s + L, b)) for s in range(a, b, L))
            return
        pre = keys[a:b] >> np.uint64(3 * (20 - lev))
        cuts = [a] + (np.nonzero(pre[1:] != pre[:-1])[0] + 1 + a).tolist() + [b]
        for u, v in zip(cuts[:-1], cuts[1:]):
            split(u, v, lev + 1)

    split(0, keys.shape[0], 0)
    return out


def support_boxes(xyz_m, tri_m, cl):
    """(lo[nc, 3], hi[nc, 3]) of each cluster's support (Morton numbering)."""
    nc = len(cl)
    owner = np.empty(xyz_m.shape[0], dtype=np.int64)
    for c, (a, b) in enumerate(cl):
        owner[a:b] = c
    lo = np.full((nc, 3), np.inf)
    hi = np.full((nc, 3), -np.inf)
    for e in range(tri_m.shape[0]):
        pts = xyz_m[tri_m[e]]
        for c in set(owner[tri_m[e]].tolist()):
            lo[c] = np.minimum(lo[c], pts.min(axis=0))
            hi[c] = np.maximum(hi[c], pts.max(axis=0))
    return lo, hi


def box_dist(lo1, hi1, lo2, hi2):
    gap = np.maximum(0.0, np.maximum(lo1 - hi2, lo2 - hi1))
    return float(np.sqrt(np.sum(gap * gap)))


def admissibility(lo, hi, eta):
    """Boolean [nc, nc] matrix of admissible cluster pairs."""
    nc = lo.shape[0]
    diam = np.linalg.norm(hi - lo, axis=1)
    adm = np.zeros((nc, nc), dtype=bool)
    for t in range(nc):
        for s in range(nc):
            if t == s:
                continue
            d = box_dist(lo[t], hi[t], lo[s], hi[s])
            adm[t, s] = d > 0 and max(diam[t], diam[s]) <= eta * d
    return adm


def aca(A, eps, rmax):
    """Adaptive cross approximation with partial pivoting of a complex
    matrix: (U[m, k], V[n, k]) with A ~ U V^T, or None when |u_k| |v_k| <=
    eps |S_k|_F is not met within rmax terms.

    Row pivots: the first row, then the largest entry of the last column
    residual among unused rows; column pivot: the largest entry of the row
    residual.  A row whose residual vanishes is marked used and the next
    unused row (lowest index) is tried instead."""
    m, n = A.shape
    us, vs = [], []
    used = np.zeros(m, dtype=bool)
    s2 = 0.0
    i = 0
    while len(us) < rmax:
        row = A[i, :] - sum((u[i] * v for u, v in zip(us, vs)), np.zeros(n, dtype=A.dtype))
        used[i] = True
        j = int(np.argmax(np.abs(row)))
        if np.abs(row[j]) == 0.0:
            free = np.where(~used)[0]
            if free.size == 0:
                return np.array(us).T.reshape(m, -1), np.array(vs).T.reshape(n, -1)
            i = int(free[0])
            continue
        v = row / row[j]
        u = A[:, j] - sum((vv[j] * uu for uu, vv in zip(us, vs)), np.zeros(m, dtype=A.dtype))
        cross = sum(2.0 * np.real(np.vdot(uu, u) * np.vdot(vv, v)) for uu, vv in zip(us, vs))
        nu, nv = np.linalg.norm(u), np.linalg.norm(v)
        s2 = s2 + cross + (nu * nv) ** 2
        us.append(u)
        vs.append(v)
        if nu * nv <= eps * np.sqrt(max(s2, 0.0)):
            return np.array(us).T, np.array(vs).T
        au = np.abs(u)
        au[used] = -1.0
        i = int(np.argmax(au))
        if au[i] < 0:
            return np.array(us).T, np.array(vs).T
    return None


def compress(Ks, xyz_m, tri_m, L, eta, eps, rmax, keep_all=False):
    """Compress the three Morton-ordered operator blocks (each [2nn, 2nn]).

    Returns dict(cl, adm, tiles) with tiles[(o, t, s)] = ("dense", A) or
    ("lowrank", U, V).  keep_all keeps every converged approximation low-rank
    even when it stores more than the dense tile (exercises small meshes)."""
    cl = clusters(node_keys(xyz_m), L)
    lo, hi = support_boxes(xyz_m, tri_m, cl)
    adm = admissibility(lo, hi, eta)
    tiles = {}
    for o, K in enumerate(Ks):
        for t, (a, b) in enumerate(cl):
            for s, (c, d) in enumerate(cl):
                A = K[2 * a:2 * b, 2 * c:2 * d]
                if adm[t, s]:
                    r = aca(A, eps, rmax)
                    if r is not None and (keep_all or r[0].shape[1] * (A.shape[0] + A.shape[1]) < A.size):
                        tiles[(o, t, s)] = ("lowrank", r[0], r[1])
                        continue
                tiles[(o, t, s)] = ("dense", A.copy())
    return dict(cl=cl, adm=adm, tiles=tiles, lo=lo, hi=hi)


def expand(C, o, n2):
    """Dense [n2, n2] matrix of operator block o of a compressed operator."""
    out = np.zeros((n2, n2), dtype=np.complex128)
    for t, (a, b) in enumerate(C["cl"]):
        for s, (c, d) in enumerate(C["cl"]):
            tile = C["tiles"][(o, t, s)]
            out[2 * a:2 * b, 2 * c:2 * d] = tile[1] if tile[0] == "dense" else tile[1] @ tile[2].T
    return out


def assemble(P, C, node_order):
    """The full Morton-ordered system matrix of a compressed operator: the
    expanded blocks with the exact (local) mass matrix, as galerkin.assemble."""
    from . import galerkin, solver
    n2 = 2 * P.nn
    p = solver.permute_unknowns(node_order)
    inv = np.empty_like(p)
    inv[p] = np.arange(p.shape[0])
    # expanded blocks back in the caller's order, then the oracle's assembly
    one = inv[:n2]
    Ks = [expand(C, o, n2)[np.ix_(one, one)] for o in range(3)]
    return galerkin.assemble(P, Ks[0], Ks[1], Ks[2], galerkin.mass_matrix(P))


def memory(C):
    """(stored complex entries, entries of the dense blocks)."""
    stored = 0
    for tile in C["tiles"].values():
        stored += tile[1].size if tile[0] == "dense" else tile[1].size + tile[2].size
    n2 = 2 * C["cl"][-1][1]
    return stored, 3 * n2 * n2
