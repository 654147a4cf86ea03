"""GPU parity of the multi-right-hand-side path: the complex GEMM on the
matrix cores (every FP32 tile shape, the FP64 variants) against the
oracle's plain product, and the block GMRES solve against dense LU of the
oracle's operator.

Tolerances:
  FP32 GEMM: 1e-5 of sum_k |a||b| per entry (FP32 products and sums over
             at most a few hundred terms: a few 1e-7 in practice);
  FP64 GEMM: 1e-13 of the same bound;
  block solve: FP64 operator 1e-9 relative to the LU solution of the
             oracle's Z at tol 1e-12; MIXED operator (complex64 storage, FP32
             far pairs: Z itself differs by ~1e-7) 1e-5, and 1e-9 against
             single-right-hand-side solves of the same operator.
"""
import numpy as np
import pytest

from oracle import core, galerkin, solver
from workloads import icosphere_p2, uv_sphere_p2
from workloads.configs import planewave_set

pytestmark = pytest.mark.gpu


def _mbem():
    from paper_2604_21181_amd import mbem
    return mbem


@pytest.fixture(scope="module")
def ctx():
    mbem = _mbem()
    c = mbem.mbem_ctx_create(0)
    yield c
    mbem.mbem_ctx_destroy(c)


def _rand(rng, shape, dtype):
    import torch
    a = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    return torch.as_tensor(a.astype(dtype), device="cuda")


# (M, Nb, K, padding of the leading dimensions): ragged M, Nb and K, a
# K tail shorter than one staging step, single rows and columns
SHAPES = [(300, 70, 257, 3), (64, 32, 8, 0), (129, 1, 1, 1), (5, 200, 40, 2), (1, 1, 3, 1)]


@pytest.mark.parametrize("cfg", range(6))
def test_cgemm_fp32_every_tile_shape(ctx, cfg):
    import torch
    mbem = _mbem()
    rng = np.random.default_rng(10 + cfg)
    for M, Nb, K, pad in SHAPES:
        lda = K + pad + ((K + pad) % 2)          # even leading dimensions
        Af = _rand(rng, (M, lda), np.complex64)
        Bf = _rand(rng, (Nb, lda), np.complex64)
        Cf = torch.zeros((Nb, M + 3), dtype=torch.complex64, device="cuda")
        A, B, Cv = Af[:, :K], Bf[:, :K], Cf[:, :M]
        mbem.mbem_cgemm(ctx, 0, False, A, B, Cv, config=cfg)
        An, Bn = A.cpu().numpy(), B.cpu().numpy()
        ref = solver.cgemm_nt(An, Bn)
        bound = np.abs(Bn).astype(np.float64) @ np.abs(An).astype(np.float64).T
        got = Cf.cpu().numpy()
        assert np.all(np.abs(got[:, :M] - ref) <= 1e-5 * bound + 1e-30), (M, Nb, K)
        assert np.all(got[:, M:] == 0), "wrote outside the output"


@pytest.mark.parametrize("dtype,conj", [(1, False), (1, True), (2, False), (2, True)])
def test_cgemm_fp64(ctx, dtype, conj):
    import torch
    mbem = _mbem()
    rng = np.random.default_rng(20 + dtype + 2 * conj)
    for M, Nb, K, pad in SHAPES:
        A = _rand(rng, (M, K + pad), np.complex64 if dtype == 2 else np.complex128)[:, :K]
        B = _rand(rng, (Nb, K + pad), np.complex128)[:, :K]
        Cf = torch.zeros((Nb, M + 1), dtype=torch.complex128, device="cuda")
        mbem.mbem_cgemm(ctx, dtype, conj, A, B, Cf[:, :M])
        An, Bn = A.cpu().numpy(), B.cpu().numpy()
        ref = solver.cgemm_nt(An, Bn, conj)
        bound = np.abs(Bn) @ np.abs(An).astype(np.float64).T
        got = Cf.cpu().numpy()
        assert np.all(np.abs(got[:, :M] - ref) <= 1e-13 * bound), (M, Nb, K)
        assert np.all(got[:, M:] == 0)


def test_cgemm_rejects_bad_operands(ctx):
    import torch
    mbem = _mbem()
    A = torch.zeros((4, 7), dtype=torch.complex64, device="cuda")   # odd lda
    B = torch.zeros((2, 8), dtype=torch.complex64, device="cuda")
    Cm = torch.zeros((2, 4), dtype=torch.complex64, device="cuda")
    with pytest.raises(mbem.MbemError) as e:
        mbem.mbem_cgemm(ctx, 0, False, A, B[:, :7], Cm)
    assert e.value.code == mbem.MBEM_EINVAL
    with pytest.raises(mbem.MbemError):
        mbem.mbem_cgemm(ctx, 0, True, B, B, Cm[:, :2])    # conj needs FP64


MESHES = {
    "sphere80": (lambda: icosphere_p2(80), 3.0, 6.0),
    "uv90_lossy": (lambda: uv_sphere_p2(9, 6, (1.0, 1.0, 1.3)), 2.0, 3.0 + 0.5j),
}


@pytest.fixture(scope="module", params=list(MESHES))
def case(request):
    mesh, k0, eps = MESHES[request.param]
    xyz, tri = mesh()
    print(f"\n[block case {request.param}]", flush=True)
    P = galerkin.Problem(xyz, tri, k0, eps)
    K = core.fill(xyz, tri, P.phys)
    Z = galerkin.assemble(P, *K, galerkin.mass_matrix(P))
    khat, pol = planewave_set(8, seed=3)
    B = galerkin.planewave_rhs(P, khat, pol).T          # [16, N]
    X = solver.solve_columns(Z, B)
    return dict(xyz=xyz, tri=tri, k0=k0, eps=eps, khat=khat, pol=pol, X=X)


def _solver(case, prec):
    mbem = _mbem()
    return mbem.Solver(case["xyz"], case["tri"], case["k0"], case["eps"], precision=prec)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("block", [4, 16])
def test_block_solve_matches_lu(case, prec, block):
    mbem = _mbem()
    S = _solver(case, mbem.MBEM_FP64 if prec == "fp64" else mbem.MBEM_MIXED)
    try:
        S.fill()
        S.precond_setup(100)
        b = S.rhs(case["khat"], case["pol"])
        x, st, code = S.solve_block(b, 1e-12, block=block)
        assert code == 0 and st.rel_resid <= 1e-12 and st.block == block
        xo = case["X"][:, S.perm]
        xg = x.cpu().numpy()
        err = np.linalg.norm(xg - xo, axis=1) / np.linalg.norm(xo, axis=1)
        assert err.max() < (1e-9 if prec == "fp64" else 1e-5), err.max()
    finally:
        S.close()


def test_block_solve_without_preconditioner_and_every_tile_shape(case):
    mbem = _mbem()
    S = _solver(case, mbem.MBEM_MIXED)
    try:
        S.fill()
        b = S.rhs(case["khat"][:8], case["pol"][:8])
        xo = case["X"][:8][:, S.perm]
        for cfg in range(mbem.GEMM_CONFIGS):
            x, st, code = S.solve_block(b, 1e-11, block=8, gemm_config=cfg, maxit=150)
            assert code == 0 and st.gemm_config == cfg
            err = np.abs(x.cpu().numpy() - xo).max() / np.abs(xo).max()
            assert err < 1e-5, (cfg, err)
            if cfg == 0:
                x0 = x
            else:   # every tile shape: the same solution of the same operator
                d = (x - x0).abs().max() / x0.abs().max()
                assert float(d) < 1e-9, (cfg, float(d))
    finally:
        S.close()


def test_block_solve_equals_single_rhs(case):
    import torch
    mbem = _mbem()
    S = _solver(case, mbem.MBEM_MIXED)
    try:
        S.fill()
        S.precond_setup(50)
        b = S.rhs(case["khat"], case["pol"])
        best, ms = S.gemm_autotune(16, reps=2)
        assert 0 <= best < mbem.GEMM_CONFIGS and np.all(ms > 0)
        xb, st, code = S.solve_block(b, 1e-11)
        assert code == 0 and st.gemm_config == best and st.block == 16
        for c in (0, 7, 15):
            xs, sst, scode = S.solve(b[c], tol=1e-11, maxit=300, inner_tol=1e-6)
            assert scode == 0
            d = torch.linalg.norm(xb[c] - xs[0]) / torch.linalg.norm(xs[0])
            assert float(d) < 1e-9
    finally:
        S.close()


def test_block_solve_rejects_bad_input(case):
    import torch
    mbem = _mbem()
    S = _solver(case, mbem.MBEM_MIXED)
    try:
        S.fill()
        b = S.rhs(case["khat"], case["pol"])
        with pytest.raises(mbem.MbemError) as e:
            S.solve_block(b, 1e-10, block=5)          # does not divide 16
        assert e.value.code == mbem.MBEM_EINVAL
        b2 = b.clone()
        b2[3].zero_()
        with pytest.raises(mbem.MbemError) as e:
            S.solve_block(b2, 1e-10)
        assert e.value.code == mbem.MBEM_EINVAL
        torch.cuda.synchronize()
    finally:
        S.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_block_solve_128_rhs_full_blocks_every_tile_shape(case, prec):
    """128 right-hand sides (64 seeded directions x 2 polarisations, the
    shape of the multi-RHS workload) in blocks of p = 32 columns, the
    largest block the solve stages in LDS, for every FP32 tile shape,
    against the LU solutions of the oracle's operator."""
    mbem = _mbem()
    khat, pol = planewave_set(64, seed=0)
    P = galerkin.Problem(case["xyz"], case["tri"], case["k0"], case["eps"])
    K = core.fill(case["xyz"], case["tri"], P.phys)
    Z = galerkin.assemble(P, *K, galerkin.mass_matrix(P))
    X = solver.solve_columns(Z, galerkin.planewave_rhs(P, khat, pol).T)      # [128, N]
    S = _solver(case, mbem.MBEM_FP64 if prec == "fp64" else mbem.MBEM_MIXED)
    try:
        S.fill()
        S.precond_setup(100)
        b = S.rhs(khat, pol)
        xo = X[:, S.perm]
        x0 = None
        for cfg in range(mbem.GEMM_CONFIGS):
            x, st, code = S.solve_block(b, 1e-12, block=32, gemm_config=cfg)
            assert code == 0 and st.block == 32 and st.gemm_config == cfg and st.rel_resid <= 1e-12
            xg = x.cpu().numpy()
            err = np.linalg.norm(xg - xo, axis=1) / np.linalg.norm(xo, axis=1)
            assert err.max() < (1e-9 if prec == "fp64" else 1e-5), (cfg, err.max())
            if x0 is None:
                x0 = xg
            else:
                d = np.linalg.norm(xg - x0, axis=1) / np.linalg.norm(x0, axis=1)
                assert d.max() < 1e-10, (cfg, d.max())
    finally:
        S.close()
