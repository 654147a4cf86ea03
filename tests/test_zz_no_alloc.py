"""The allocation-free product (mbem_matvec_noalloc) against mbem_matvec.

For callers that cannot allocate: the partial sums live in the library's
file-scope device array.  Two operators in a row, the second smaller than
the first (the array keeps the first call's contents), FP64 and mixed with
the FP64 near store, one and two right-hand sides: every product equals the
allocating entry point's bit for bit (same kernels, same operands).
"""
import numpy as np
import pytest

from workloads import icosphere_p2

pytestmark = pytest.mark.gpu


def _product_pair(mbem, S, nrhs, seed):
    import torch
    rng = np.random.default_rng(seed)
    x = torch.as_tensor(rng.normal(size=(nrhs, S.N)) + 1j * rng.normal(size=(nrhs, S.N)), device=S.device)
    y_ref = torch.empty_like(x)
    mbem.mbem_matvec(S.ctx, S.op, x, y_ref, nrhs)
    torch.cuda.synchronize()
    y = torch.full_like(x, complex(float("nan"), 0.0))
    mbem.mbem_matvec_noalloc(S.ctx, S.op, x, y, nrhs)
    torch.cuda.synchronize()
    return y.cpu().numpy(), y_ref.cpu().numpy()


def test_noalloc_matvec_matches_matvec():
    from paper_2604_21181_amd import mbem
    print("\n[noalloc matvec: sphere320 then sphere80]", flush=True)
    for prec, store in ((mbem.MBEM_FP64, False), (mbem.MBEM_MIXED, True)):
        for nt, nrhs in ((320, 2), (80, 1)):
            xyz, tri = icosphere_p2(nt)
            S = mbem.Solver(xyz, tri, 2.0, 4.0, precision=prec, near_store=store)
            try:
                S.fill()
                y, y_ref = _product_pair(mbem, S, nrhs, seed=nt)
                assert np.isfinite(y).all()
                assert np.array_equal(y, y_ref), (prec, nt, np.abs(y - y_ref).max())
            finally:
                S.close()


def test_noalloc_matvec_rejects_null_arguments():
    import ctypes as C
    from paper_2604_21181_amd import mbem
    L = mbem.lib()
    assert L.mbem_matvec_noalloc(None, None, None, 1, None) == mbem.MBEM_EINVAL
