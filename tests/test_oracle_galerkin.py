"""Pins of the oracle's Galerkin system, solver and post-processing."""
import numpy as np
import pytest

import oracle
from oracle import core, galerkin, mie, solver
from workloads import icosphere_p2
from workloads.configs import cut_plane_directions

KH = np.array([0.0, 0.0, 1.0])
POL = np.array([1.0, 0.0, 0.0], dtype=np.complex128)


@pytest.fixture(scope="module")
def c1():
    xyz, tri = icosphere_p2(80)
    P = galerkin.Problem(xyz, tri, 1.0, 4.0)
    x, K, M = oracle.solve_dense(P, KH[None], POL[None])
    return P, x[:, 0], K, M


def _S(B):
    """S_ab(e,f)_ij = B(N_i t_a, N_j t_b) from a K1 block, using
    s_1 = -t_2, s_2 = t_1 (Sec. 4.1): K1_1b = -S_2b, K1_2b = S_1b."""
    K = B[:, :, 0:4].reshape(6, 6, 2, 2)
    s = np.zeros((2, 2, 6, 6), complex)
    s[1] = -np.moveaxis(K[:, :, 0, :], 2, 0)
    s[0] = np.moveaxis(K[:, :, 1, :], 2, 0)
    return s


def _pair_class(tri, e, f):
    return len(set(tri[e, :3]) & set(tri[f, :3]))


def test_galerkin_symmetry_regular_vertex_coincident(c1):
    """The kernel s_a(x).[D0 I + H_diff(x,y)].t_b(y) is a symmetric bilinear
    form, so S_ab(e,f) = S_ba(f,e)^T.  The regular rule and the coincident /
    common-vertex Sauter-Schwab rules are symmetric under x <-> y, so these
    pairs must satisfy it to rounding."""
    P, x, K, M = c1
    rng = np.random.default_rng(5)
    pairs = {0: [], 1: [], 3: []}
    for e in range(P.nt):
        for f in range(P.nt):
            c = _pair_class(P.tri6, e, f)
            if c in pairs:
                pairs[c].append((e, f))
    for c, lst in pairs.items():
        for k in rng.choice(len(lst), size=min(12, len(lst)), replace=False):
            e, f = lst[k]
            a = _S(core.pair_block(P.xyz, P.tri6, P.phys, e, f))
            b = _S(core.pair_block(P.xyz, P.tri6, P.phys, f, e))
            d = np.abs(a - np.transpose(b, (1, 0, 3, 2))).max()
            assert d <= 1e-13 * np.abs(a).max(), (c, e, f, d)


def test_galerkin_symmetry_edge_pairs_converge(c1):
    """Common-edge Sauter-Schwab regions are not mirror images, so edge pairs
    are symmetric only to the rule's accuracy: on pairs whose twelve nodes
    share one reference axis (smooth frames) the asymmetry falls below 1e-8
    at 8 points per dimension."""
    P, x, K, M = c1
    n = core.nodal_frames(P.xyz, P.tri6)[0]
    polar = np.abs(n[:, 2]) > 0.9
    checked = 0
    for e in range(P.nt):
        for f in range(P.nt):
            if _pair_class(P.tri6, e, f) != 2:
                continue
            nodes = np.concatenate([P.tri6[e], P.tri6[f]])
            if polar[nodes].any() and not polar[nodes].all():
                continue
            a = _S(core.pair_block(P.xyz, P.tri6, P.phys, e, f, nss=8))
            b = _S(core.pair_block(P.xyz, P.tri6, P.phys, f, e, nss=8))
            d = np.abs(a - np.transpose(b, (1, 0, 3, 2))).max()
            assert d <= 1e-8 * np.abs(a).max(), (e, f, d)
            checked += 1
            if checked >= 10:
                return
    assert checked > 0


def test_assembled_symmetries(c1):
    """K1_12 = K1_12^T, K1_21 = K1_21^T, K1_22 = -K1_11^T hold on every entry
    that no common-edge pair touches across a reference-axis switch; check
    the regular part exactly by removing all singular-pair contributions."""
    P, x, K, M = c1
    n2 = 2 * P.nn
    Kr = np.zeros((n2, n2), complex)
    rng = np.random.default_rng(7)
    es = rng.choice(P.nt, 20, replace=False)
    for e in es:
        for f in es:
            if _pair_class(P.tri6, e, f) != 0:
                continue
            B = core.pair_block(P.xyz, P.tri6, P.phys, e, f)
            for i in range(6):
                for j in range(6):
                    Kr[2 * P.tri6[e, i]:2 * P.tri6[e, i] + 2,
                       2 * P.tri6[f, j]:2 * P.tri6[f, j] + 2] += B[i, j, 0:4].reshape(2, 2)
    s = np.abs(Kr).max()
    A = Kr[0::2, 1::2]
    assert np.abs(A - A.T).max() <= 1e-13 * s
    A = Kr[1::2, 0::2]
    assert np.abs(A - A.T).max() <= 1e-13 * s
    assert np.abs(Kr[1::2, 1::2] + Kr[0::2, 0::2].T).max() <= 1e-13 * s


def test_fill_equals_pair_block_assembly(c1):
    """The dense fill is the plain sum of pair blocks over element pairs."""
    P, x, K, M = c1
    for (I, J) in [(0, 0), (3, 50), (100, 7), (161, 161)]:
        ent = core.entries(P.xyz, P.tri6, P.phys, [I], [J])[0]
        for o in range(3):
            assert np.abs(K[o][2 * I:2 * I + 2, 2 * J:2 * J + 2] - ent[o]).max() < 1e-17 + 1e-14 * np.abs(ent[o]).max()


def test_zero_contrast(sphere80):
    """eps_r = mu_r = 1: every kernel difference vanishes, Z = [[0,M],[M,0]],
    and the L2-projected incident currents radiate (almost) nothing outside
    (extinction theorem); the j and j_m far-field terms must cancel."""
    xyz, tri = sphere80
    P = galerkin.Problem(xyz, tri, 1.0, 1.0)
    x, K, M = oracle.solve_dense(P, KH[None], POL[None])
    for k in K:
        assert np.all(k == 0)
    r = cut_plane_directions(72)
    F = galerkin.far_field(P, x[:, 0], r)
    xj = x[:, 0].copy()
    xj[2 * P.nn:] = 0
    Fj = galerkin.far_field(P, xj, r)
    assert np.abs(F).max() < 0.02 * np.abs(Fj).max()


def test_mie_sphere80(c1):
    P, x, K, M = c1
    ce, cs, ca = galerkin.cross_sections(P, x, KH, POL)
    me, ms, _ = mie.cross_sections(1.0, 1.0, 4.0)
    assert abs(ce - me) / me < 1e-2
    assert abs(cs - ms) / ms < 6e-2
    assert abs(ca) / ce < 1e-2                   # lossless sphere
    r = cut_plane_directions()
    Fo = galerkin.far_field(P, x, r)
    Fm = mie.far_field(1.0, 1.0, 4.0, r)
    assert np.linalg.norm(Fo - Fm) / np.linalg.norm(Fm) < 3e-2


def test_mie_converges_under_refinement(c1):
    P80, x80, _, _ = c1
    xyz, tri = icosphere_p2(320)
    P = galerkin.Problem(xyz, tri, 1.0, 4.0)
    x, _, _ = oracle.solve_dense(P, KH[None], POL[None])
    r = cut_plane_directions(90)
    Fm = mie.far_field(1.0, 1.0, 4.0, r)
    e80 = np.linalg.norm(galerkin.far_field(P80, x80, r) - Fm)
    e320 = np.linalg.norm(galerkin.far_field(P, x[:, 0], r) - Fm)
    assert e320 < 0.75 * e80


def test_optical_theorem_lossy():
    """Lossy sphere: C_ext (optical theorem) = C_sca + C_abs to
    discretisation error, and C_abs > 0."""
    xyz, tri = icosphere_p2(80)
    P = galerkin.Problem(xyz, tri, 1.0, 3.0 + 0.5j)
    x, _, _ = oracle.solve_dense(P, KH[None], POL[None])
    ce, cs, ca = galerkin.cross_sections(P, x[:, 0], KH, POL)
    me, ms, ma = mie.cross_sections(1.0, 1.0, 3.0 + 0.5j)
    assert ca > 0 and abs(ca - ma) / ma < 5e-2
    assert abs(ce - cs - ca) / ce < 5e-2


def test_gmres_matches_lu_and_mbj(c1):
    P, x, K, M = c1
    no, to = solver.morton_order(P.xyz, P.tri6)
    p = solver.permute_unknowns(no)
    Z = galerkin.assemble(P, *K, M)[np.ix_(p, p)]
    b = galerkin.planewave_rhs(P, KH[None], POL[None])[:, 0][p]
    x0, it0, _ = solver.gmres(lambda v: Z @ v, b, tol=1e-11)
    bl = solver.mbj_matrices(Z, 100)
    x1, it1, _ = solver.gmres(lambda v: Z @ v, b,
                              precond=lambda v: solver.mbj_apply(bl, v, 100), tol=1e-11)
    for xs in (x0, x1):
        assert np.linalg.norm(xs - x[p]) / np.linalg.norm(x) < 1e-9
    assert it1 < it0 / 3                       # MBJ clusters the spectrum
    n = Z.shape[0]
    bl = solver.mbj_matrices(Z, n // 2)        # one block: P = Z
    _, it2, _ = solver.gmres(lambda v: Z @ v, b,
                             precond=lambda v: solver.mbj_apply(bl, v, n // 2), tol=1e-11)
    assert it2 == 1


def test_morton_order_properties(c1):
    P, *_ = c1
    no, to = solver.morton_order(P.xyz, P.tri6)
    assert sorted(no) == list(range(P.nn)) and sorted(to) == list(range(P.nt))
    lo = P.xyz.min(0)
    ext = float((P.xyz.max(0) - lo).max())
    k = solver.morton_keys(P.xyz[no], lo, ext)
    assert np.all(np.diff(k.astype(np.float64)) >= 0)
    # Z-order locality: consecutive nodes are much closer than random pairs
    d = np.linalg.norm(np.diff(P.xyz[no], axis=0), axis=1).mean()
    rnd = np.linalg.norm(P.xyz[1:] - P.xyz[:-1][::-1], axis=1).mean()
    assert d < 0.5 * rnd
