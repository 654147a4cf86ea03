"""Pins of the oracle's block linear algebra: the complex GEMM against a
brute-force triple loop and the column solve against the residual."""
import numpy as np

from oracle import solver


def test_cgemm_nt_brute_force():
    rng = np.random.default_rng(5)
    A = rng.normal(size=(5, 3)) + 1j * rng.normal(size=(5, 3))
    B = rng.normal(size=(4, 3)) + 1j * rng.normal(size=(4, 3))
    for conj in (False, True):
        C = solver.cgemm_nt(A, B, conj)
        ref = np.zeros((4, 5), dtype=complex)
        for b in range(4):
            for m in range(5):
                for k in range(3):
                    a = np.conj(A[m, k]) if conj else A[m, k]
                    ref[b, m] += a * B[b, k]
        assert np.abs(C - ref).max() < 1e-14


def test_solve_columns_residual():
    rng = np.random.default_rng(6)
    Z = rng.normal(size=(30, 30)) + 1j * rng.normal(size=(30, 30)) + 10 * np.eye(30)
    B = rng.normal(size=(7, 30)) + 1j * rng.normal(size=(7, 30))
    X = solver.solve_columns(Z, B)
    for c in range(7):
        assert np.linalg.norm(Z @ X[c] - B[c]) < 1e-13 * np.linalg.norm(B[c])
