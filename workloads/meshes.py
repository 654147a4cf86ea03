"""Closed P2 (6-node) triangle meshes of spheres, spheroids and ellipsoids.

Recipe (used for every workload):
  1. the regular icosahedron with vertices (0,+-1,+-phi), (+-1,+-phi,0),
     (+-phi,0,+-1), phi = (1+sqrt 5)/2, projected to the unit sphere;
  2. L rounds of 1->4 midpoint subdivision, new vertices projected to the
     unit sphere after each round (F = 20 * 4**L triangles);
  3. one P2 mid-edge node per edge at normalize((x_p + x_q)/2);
  4. every triangle oriented counter-clockwise seen from outside;
  5. all nodes scaled by diag(a, b, c) for spheroids and ellipsoids.

The cubed-sphere meshes (``cubesphere_p2``) replace steps 1-2 by: the
surface lattice points (i, j, k) in {0..n}^3 of a cube (some coordinate 0 or
n), mapped coordinate-wise by t -> tan(pi/4 (2t/n - 1)) (the equiangular
gnomonic map; the face coordinate becomes +-1) and projected to the unit
sphere; each of the 6 n^2 lattice squares split along its (i, j) -> (i+1,
j+1) diagonal (F = 12 n^2 triangles).  Steps 3-5 are the same.

Node order is the generation order (vertices first, then edge nodes); it is
deliberately *not* spatially sorted, so that the library's own reordering is
exercised.  Local node order of a triangle is (v0, v1, v2, m01, m12, m20).
"""
from __future__ import annotations

import math

import numpy as np


def _icosahedron():
    p = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([
        [-1, p, 0], [1, p, 0], [-1, -p, 0], [1, -p, 0],
        [0, -1, p], [0, 1, p], [0, -1, -p], [0, 1, -p],
        [p, 0, -1], [p, 0, 1], [-p, 0, -1], [-p, 0, 1],
    ], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
    ], dtype=np.int64)
    return v, f


def _orient_outward(v, f):
    a, b, c = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    s = np.einsum("ij,ij->i", np.cross(b - a, c - a), a + b + c)
    f = f.copy()
    bad = s < 0
    f[bad] = f[bad][:, [0, 2, 1]]
    return f


def _subdivide(v, f):
    verts = [row for row in v]
    cache = {}

    def mid(i, j):
        key = (min(i, j), max(i, j))
        if key not in cache:
            m = verts[i] + verts[j]
            verts.append(m / np.linalg.norm(m))
            cache[key] = len(verts) - 1
        return cache[key]

    out = []
    for a, b, c in f:
        ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
        out += [[a, ab, ca], [ab, b, bc], [ca, bc, c], [ab, bc, ca]]
    return np.array(verts), np.array(out, dtype=np.int64)


def mesh_counts(n_tris: int):
    """(n_nodes, n_unknowns) of a closed P2 surface with n_tris triangles."""
    n_nodes = 2 * n_tris + 2
    return n_nodes, 4 * n_nodes


def icosphere_p2(n_tris: int, axes=(1.0, 1.0, 1.0)):
    """Return (xyz[n_nodes,3] float64, tri6[n_tris,6] int64)."""
    levels = 0
    while 20 * 4 ** levels < n_tris:
        levels += 1
    if 20 * 4 ** levels != n_tris:
        raise ValueError(f"n_tris must be 20*4**L, got {n_tris}")
    v, f = _icosahedron()
    for _ in range(levels):
        v, f = _subdivide(v, f)
    f = _orient_outward(v, f)
    nv = v.shape[0]
    edge_id = {}
    mids = []
    tri6 = np.zeros((f.shape[0], 6), dtype=np.int64)
    for t, (a, b, c) in enumerate(f):
        tri6[t, :3] = (a, b, c)
        for k, (p, q) in enumerate(((a, b), (b, c), (c, a))):
            key = (min(p, q), max(p, q))
            if key not in edge_id:
                m = v[p] + v[q]
                mids.append(m / np.linalg.norm(m))
                edge_id[key] = nv + len(mids) - 1
            tri6[t, 3 + k] = edge_id[key]
    xyz = np.concatenate([v, np.array(mids)], axis=0)
    xyz = xyz * np.asarray(axes, dtype=np.float64)[None, :]
    assert xyz.shape[0] == mesh_counts(n_tris)[0]
    return np.ascontiguousarray(xyz), np.ascontiguousarray(tri6)


def _p2_nodes(v, f, axes):
    """Mid-edge nodes (step 3), tri6 connectivity and the scaling of step 5."""
    nv = v.shape[0]
    edge_id, mids = {}, []
    tri6 = np.zeros((f.shape[0], 6), dtype=np.int64)
    for t, (a, b, c) in enumerate(f):
        tri6[t, :3] = (a, b, c)
        for k, (p, q) in enumerate(((a, b), (b, c), (c, a))):
            key = (min(p, q), max(p, q))
            if key not in edge_id:
                m = v[p] + v[q]
                mids.append(m / np.linalg.norm(m))
                edge_id[key] = nv + len(mids) - 1
            tri6[t, 3 + k] = edge_id[key]
    xyz = np.concatenate([v, np.array(mids)], axis=0) * np.asarray(axes, dtype=np.float64)[None, :]
    return np.ascontiguousarray(xyz), np.ascontiguousarray(tri6)


def cubesphere_p2(n: int, axes=(1.0, 1.0, 1.0)):
    """Equiangular cubed sphere with n x n squares per cube face, each split
    into two triangles: 12 n^2 P2 triangles on 6 n^2 + 2 vertices, 24 n^2 + 2
    nodes in all.  n = 16 gives 3072 triangles and 6146 nodes.
    Returns (xyz[n_nodes,3] float64, tri6[n_tris,6] int64)."""
    if n < 1:
        raise ValueError("n must be positive")
    index = {}
    verts = []

    def vid(i, j, k):
        key = (i, j, k)
        if key not in index:
            q = np.tan(0.25 * math.pi * (2.0 * np.array(key, dtype=np.float64) / n - 1.0))
            verts.append(q / np.linalg.norm(q))
            index[key] = len(verts) - 1
        return index[key]

    f = []
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        for side in (0, n):
            for i in range(n):
                for j in range(n):
                    corners = []
                    for di, dj in ((0, 0), (1, 0), (1, 1), (0, 1)):
                        p = [0, 0, 0]
                        p[a], p[b], p[c] = side, i + di, j + dj
                        corners.append(vid(*p))
                    p00, p10, p11, p01 = corners
                    f += [[p00, p10, p11], [p00, p11, p01]]
    v = np.array(verts)
    f = _orient_outward(v, np.array(f, dtype=np.int64))
    xyz, tri6 = _p2_nodes(v, f, axes)
    assert xyz.shape[0] == mesh_counts(tri6.shape[0])[0]
    return xyz, tri6


def uv_sphere_p2(n_lon: int, n_lat: int, axes=(1.0, 1.0, 1.0)):
    """Latitude-longitude triangulation of the unit sphere (two poles,
    n_lat - 1 rings of n_lon vertices), P2 mid-edge nodes projected to the
    sphere, oriented outward, then scaled by diag(axes).

    n_tris = 2 n_lon (n_lat - 1); odd n_lon and even n_lat give a count
    that is not a multiple of 4, and the poles have valence n_lon.
    """
    verts = [np.array([0.0, 0.0, 1.0])]
    for k in range(1, n_lat):
        th = math.pi * k / n_lat
        for j in range(n_lon):
            ph = 2 * math.pi * j / n_lon
            verts.append(np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph),
                                   math.cos(th)]))
    verts.append(np.array([0.0, 0.0, -1.0]))
    v = np.array(verts)
    south = v.shape[0] - 1

    def ring(k, j):
        return 1 + (k - 1) * n_lon + (j % n_lon)

    f = []
    for j in range(n_lon):
        f.append([0, ring(1, j), ring(1, j + 1)])
        f.append([south, ring(n_lat - 1, j + 1), ring(n_lat - 1, j)])
    for k in range(1, n_lat - 1):
        for j in range(n_lon):
            a, b = ring(k, j), ring(k, j + 1)
            c, d = ring(k + 1, j), ring(k + 1, j + 1)
            f += [[a, c, d], [a, d, b]]
    f = _orient_outward(v, np.array(f, dtype=np.int64))
    return _p2_nodes(v, f, axes)
