"""Pins of the oracle's block low-rank compression (CPU).

* ACA recovers an exactly low-rank matrix (to rounding, with at most one
  extra term) and comes close to the optimal (SVD) rank on a smooth kernel,
  at the requested accuracy.
* Zero rows and an all-zero tile are handled (skipped / rank 0).
* The tiles partition the operator exactly once; an admissible cluster pair
  has disjoint supports (no element touches both), so every interaction in it
  is a regular pair, and meets the eta condition.
* The compressed operator of a sphere is within a small multiple of eps of
  the dense one, its near tiles are exact, and its solve gives the dense far
  field to the accuracy eps allows.
"""
import numpy as np
import pytest

from oracle import blr, core, galerkin, solver
from workloads import icosphere_p2


def test_aca_recovers_exact_low_rank():
    rng = np.random.default_rng(0)
    for r, (m, n) in ((1, (30, 50)), (5, (60, 40)), (12, (80, 90))):
        U = rng.normal(size=(m, r)) + 1j * rng.normal(size=(m, r))
        V = rng.normal(size=(n, r)) + 1j * rng.normal(size=(n, r))
        A = U @ V.T
        Ua, Va = blr.aca(A, 1e-12, 40)
        assert Ua.shape[1] <= r + 1
        assert np.abs(Ua @ Va.T - A).max() <= 1e-12 * np.abs(A).max()


@pytest.mark.parametrize("eps", [1e-4, 1e-6, 1e-8])
def test_aca_near_optimal_on_a_smooth_kernel(eps):
    rng = np.random.default_rng(1)
    x = rng.uniform(-1, 1, size=(90, 3))
    y = rng.uniform(-1, 1, size=(70, 3)) + np.array([5.0, 0, 0])
    R = np.linalg.norm(x[:, None] - y[None], axis=2)
    A = np.exp(2j * R) / R
    Ua, Va = blr.aca(A, eps, 80)
    err = np.linalg.norm(Ua @ Va.T - A) / np.linalg.norm(A)
    s = np.linalg.svd(A, compute_uv=False)
    tail = np.sqrt(np.cumsum((s ** 2)[::-1])[::-1]) / np.linalg.norm(s)
    r_opt = int(np.argmax(tail <= eps)) if np.any(tail <= eps) else len(s)
    assert err <= 5 * eps
    assert Ua.shape[1] <= 2 * r_opt + 5


def test_aca_zero_rows_and_zero_tile():
    rng = np.random.default_rng(2)
    A = (rng.normal(size=(20, 3)) @ rng.normal(size=(3, 25))).astype(np.complex128)
    A[:4] = 0.0                                   # the first row pivots vanish
    Ua, Va = blr.aca(A, 1e-10, 20)
    assert np.abs(Ua @ Va.T - A).max() <= 1e-12 * np.abs(A).max()
    Uz, Vz = blr.aca(np.zeros((6, 7), dtype=np.complex128), 1e-6, 5)
    assert Uz.shape == (6, 0) and Vz.shape == (7, 0)
    # no convergence within rmax
    assert blr.aca(rng.normal(size=(30, 30)).astype(np.complex128), 1e-12, 5) is None


def _morton(xyz, tri):
    no, _ = solver.morton_order(xyz, tri)
    rank = np.empty_like(no)
    rank[no] = np.arange(no.shape[0])
    return no, xyz[no], rank[tri]


@pytest.mark.parametrize("L,eta", [(16, 3.0), (12, 2.0), (24, 1.5)])
def test_partition_and_admissibility(L, eta):
    xyz, tri = icosphere_p2(320)
    no, xyz_m, tri_m = _morton(xyz, tri)
    keys = blr.node_keys(xyz_m)
    cl = blr.clusters(keys, L)
    assert cl[0][0] == 0 and cl[-1][1] == xyz.shape[0]
    assert all(a[1] == b[0] for a, b in zip(cl[:-1], cl[1:]))
    assert all(0 < b - a <= L for a, b in cl)
    # each cluster is an octree cell (or a piece of a finest cell): its keys
    # share a prefix that no neighbouring cluster's keys extend
    for a, b in cl:
        common = 0
        for lev in range(22):
            sh = np.uint64(3 * (21 - lev))
            if np.all((keys[a:b] >> sh) == (keys[a] >> sh)):
                common = lev
        sh = np.uint64(3 * (21 - common))
        inside = (keys >> sh) == (keys[a] >> sh)
        # the cell of that prefix holds more than L nodes unless it is the cluster
        assert inside.sum() == b - a or inside.sum() > L
    lo, hi = blr.support_boxes(xyz_m, tri_m, cl)
    adm = blr.admissibility(lo, hi, eta)
    assert not np.any(np.diag(adm)) and adm.sum() > 0
    owner = np.empty(xyz.shape[0], dtype=np.int64)
    for c, (a, b) in enumerate(cl):
        owner[a:b] = c
    touch = [set(owner[t].tolist()) for t in tri_m]
    for t, s in zip(*np.nonzero(adm)):
        # no element touches both clusters: every interaction is regular
        assert not any(t in ts and s in ts for ts in touch)
        d = blr.box_dist(lo[t], hi[t], lo[s], hi[s])
        assert d > 0 and max(np.linalg.norm(hi[t] - lo[t]), np.linalg.norm(hi[s] - lo[s])) <= eta * d
        # every node of every element touching a cluster lies in its box
        for c in (t, s):
            pts = xyz_m[np.unique(tri_m[[c in ts for ts in touch]])]
            assert np.all(pts >= lo[c] - 1e-15) and np.all(pts <= hi[c] + 1e-15)


@pytest.fixture(scope="module")
def sphere320():
    xyz, tri = icosphere_p2(320)
    P = galerkin.Problem(xyz, tri, 3.0, 2.25)
    K = core.fill(xyz, tri, P.phys)
    no, xyz_m, tri_m = _morton(xyz, tri)
    p = solver.permute_unknowns(no)[: 2 * xyz.shape[0]]
    Km = [k[np.ix_(p, p)] for k in K]
    return P, K, Km, no, xyz_m, tri_m


def test_compressed_operator_error(sphere320):
    P, K, Km, no, xyz_m, tri_m = sphere320
    eps = 1e-6
    C = blr.compress(Km, xyz_m, tri_m, 16, 3.0, eps, 64, keep_all=True)
    n_lr = sum(1 for v in C["tiles"].values() if v[0] == "lowrank")
    assert n_lr > 3000
    for o in range(3):
        E = blr.expand(C, o, Km[o].shape[0])
        assert np.linalg.norm(E - Km[o]) <= 10 * eps * np.linalg.norm(Km[o])
        for (oo, t, s), tile in C["tiles"].items():
            if oo == o and tile[0] == "dense":
                (a, b), (c, d) = C["cl"][t], C["cl"][s]
                assert np.array_equal(E[2 * a:2 * b, 2 * c:2 * d], Km[o][2 * a:2 * b, 2 * c:2 * d])


def test_compressed_solve_far_field(sphere320):
    P, K, Km, no, xyz_m, tri_m = sphere320
    kh, pol = np.array([0, 0, 1.0]), np.array([1.0, 0, 0], dtype=np.complex128)
    M = galerkin.mass_matrix(P)
    b = galerkin.planewave_rhs(P, kh, pol)[:, 0]
    x = np.linalg.solve(galerkin.assemble(P, *K, M), b)
    rdir = np.array([[np.sin(t), 0, np.cos(t)] for t in np.linspace(0, np.pi, 19)])
    F = galerkin.far_field(P, x, rdir)
    for eps, tol in ((1e-4, 2e-3), (1e-6, 2e-5)):
        C = blr.compress(Km, xyz_m, tri_m, 16, 3.0, eps, 64, keep_all=True)
        xc = np.linalg.solve(blr.assemble(P, C, no), b)
        Fc = galerkin.far_field(P, xc, rdir)
        assert np.linalg.norm(Fc - F) / np.linalg.norm(F) <= tol, eps
