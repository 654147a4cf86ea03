"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The oracle's C core and the library's host preprocessing (mesh validation,
the double Morton permutation of Sec. 5, singular-pair lists of Sec. 4.2,
mass pattern, trial chunks, colour classes) are rebuilt with gcc / g++
and -fsanitize=address,undefined into two small drivers under
tests/sanitize/, run on P2 meshes, and must exit cleanly: any heap or stack
overflow, use after free, leak, signed overflow, misaligned or out-of-range
access aborts the driver with a report.  The sanitized builds must also give
the same results as the production builds: the oracle's dense blocks and
nodal frames equal those of liboracle.so, the host permutation equals the
library's (mbem_morton_order).
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import core, galerkin
from workloads import icosphere_p2, uv_sphere_p2

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2604_21181_amd", "csrc")
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
       "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:strict_string_checks=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")

MESHES = {"ico80": lambda: icosphere_p2(80),
          "uv54_ellipsoid": lambda: uv_sphere_p2(9, 6, (1.0, 1.0, 1.3))}


def _have(tool):
    return shutil.which(tool) is not None


@pytest.fixture(scope="module")
def drivers(tmp_path_factory):
    if not (_have("gcc") and _have("g++")):
        pytest.skip("gcc / g++ not available")
    d = tmp_path_factory.mktemp("san")
    oracle_bin = str(d / "oracle_driver")
    subprocess.run(["gcc", "-std=c11", *SAN, "-o", oracle_bin,
                    os.path.join(HERE, "sanitize", "oracle_driver.c"),
                    os.path.join(ROOT, "oracle", "mbem_oracle.c"), "-lm"],
                   check=True, capture_output=True)
    host_bin = str(d / "host_driver")
    subprocess.run(["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    "-I" + CSRC, "-o", host_bin, os.path.join(HERE, "sanitize", "host_driver.cpp"),
                    os.path.join(CSRC, "host_mesh.cpp")],
                   check=True, capture_output=True)
    return d, oracle_bin, host_bin


def _write_mesh(path, xyz, tri, phys=None):
    with open(path, "wb") as f:
        np.array([xyz.shape[0], tri.shape[0]], dtype=np.int64).tofile(f)
        np.ascontiguousarray(xyz, dtype=np.float64).tofile(f)
        np.ascontiguousarray(tri, dtype=np.int64).tofile(f)
        if phys is not None:
            np.asarray(phys, dtype=np.float64).tofile(f)


def _run(binary, inp, out):
    r = subprocess.run([binary, inp, out], env=ENV, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr[-4000:]


@pytest.mark.parametrize("mesh", list(MESHES))
def test_host_preprocessing_clean_and_equal(drivers, mesh):
    d, _, host_bin = drivers
    xyz, tri = MESHES[mesh]()
    inp, out = str(d / f"{mesh}.mesh"), str(d / f"{mesh}.host")
    _write_mesh(inp, xyz, tri)
    _run(host_bin, inp, out)
    res = np.fromfile(out, dtype=np.int64)
    nn, nt = xyz.shape[0], tri.shape[0]
    no, to, ns = res[:nn], res[nn:nn + nt], res[nn + nt:]
    assert ns.shape == (4,) and ns.sum() > 0
    from paper_2604_21181_amd import mbem
    lno, lto = mbem.mbem_morton_order(xyz, tri)
    assert np.array_equal(no, lno) and np.array_equal(to, lto)


@pytest.mark.parametrize("variant,frame", [(0, 0), (1, 0), (0, 1)])
def test_oracle_core_clean_and_equal(drivers, variant, frame):
    d, oracle_bin, _ = drivers
    xyz, tri = icosphere_p2(20)
    P = galerkin.Problem(xyz, tri, 2.0, 3.0 + 0.2j, variant=variant, frame=frame)
    inp, out = str(d / f"o{variant}{frame}.mesh"), str(d / f"o{variant}{frame}.out")
    _write_mesh(inp, xyz, tri, P.phys)
    _run(oracle_bin, inp, out)
    n2 = 2 * xyz.shape[0]
    raw = np.fromfile(out, dtype=np.float64)
    Ks = raw[:6 * n2 * n2].view(np.complex128).reshape(3, n2, n2)
    frames = raw[6 * n2 * n2:].reshape(-1, 3, 3).transpose(1, 0, 2)     # (n, t1, t2) per node
    K = core.fill(xyz, tri, P.phys, nss=3, nthreads=1)
    for o in range(3):
        scale = np.abs(K[o]).max()
        assert np.abs(Ks[o] - K[o]).max() <= 1e-13 * scale, o
    assert np.abs(frames - core.nodal_frames(xyz, tri)).max() <= 1e-14
