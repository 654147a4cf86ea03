"""Benchmark of the nodal P2 Mueller hot path on one MI355X.

Workload (default): the 1280-triangle unit sphere, k_a = 5, eps_r = 2.25,
2562 nodes, N = 10248 complex unknowns, one x-polarised plane wave along
+z, 7-point regular rule, 4^4-point Sauter-Schwab rule, Morton block-Jacobi
with B = 100, GMRES to 1e-8, far field at 360 angles of the xz plane.

One step = the whole hot path, both precisions side by side:
  FP64 : fill (geometry, all pair classes, mass) -> block-Jacobi setup ->
         right-hand side -> GMRES -> far field
  MIXED: the same with FP32 far pairs / complex64 storage and FP64
         iterative refinement.
  GRADIENT: 1280-triangle ellipsoid (1, 0.8, 0.6), k_a = 3, eps_r = 3 + 0.1i:
         FP64 fill -> block-Jacobi setup -> GMRES to 1e-12 -> adjoint
         (Z^T solve, dZ/deps_r fill, reverse pass over every point pair and
         the geometry) -> sigma_ext, d sigma/d eps_r, d sigma/d(normal
         displacement) of every node.
  MULTI-RHS: the same sphere at k_a = 3, eps_r = 6 with 128 plane waves
         (64 seeded directions x 2 polarisations): mixed fill ->
         block-Jacobi setup -> 128 right-hand sides -> block GMRES (complex
         FP32 GEMM on the matrix cores, FP64 refinement) to 1e-8 -> far
         fields in the 64 incidence directions.
  PRECONDITIONER STUDY (once, after the timed steps): FP64 operators of the
         1280-triangle sphere and the 5120-triangle spheroid (1, 1, 2),
         k_a = 4, eps_r = -10 + 1i; GMRES to 1e-5 without a preconditioner
         and with Morton block-Jacobi for clusters of 50, 100, 256 and 512:
         iterations, setup and solve times.
  SPECTRUM STUDY (once): the silver-spheroid LSPR spectrum (15 x 15 x 45 nm,
         3072-triangle cubed sphere, 24584 unknowns, permittivity from the
         printed Johnson-Christy table) over the 131-wavelength grid in one
         call of the sweep entry point, FP64 and mixed: per-point refill,
         block-Jacobi (clusters of 100), GMRES to 1e-5 and cross sections;
         points per second, phase times, the extinction peak and the energy
         balance.  The preconditioner study also runs this spheroid at its
         506 nm resonance (the paper's comparison of 822 vs 18 iterations).
  COMPRESSED OPERATOR STUDY (once): the block low-rank operator (octree
         clusters of at most 512 nodes, eta = 2, cross approximation to 1e-6)
         on a 20480-triangle sphere, k_a = 5, eps_r = 2.25: 163848 unknowns,
         whose dense FP64 blocks (322 GB) exceed the device; fill and
         compression time, stored bytes, the compressed product's time and
         bandwidth, GMRES (block-Jacobi, 100) to 1e-8, cross sections and
         their energy balance.
  QUADRATURE STUDY (once): the paper's own scheme (12-point rule, Sauter-
         Schwab on the singular kernels only, 12-point remainder) against the
         default on the same sphere, FP64 and mixed: fill times and far-field
         differences.
  SPHEROID PASS (once): the 5120-triangle plasmonic spheroid (1, 1, 2),
         k_a = 4, eps_r = -10 + 1i, 40968 unknowns, block-Jacobi B = 256, one
         plane wave: FP64, mixed with the FP64 near store (the workload's
         storage) and mixed without it; fill and GMRES to 1e-6 (iterations,
         times) and to 1e-10, every far field against the FP64 one at 1e-10.
Metric: Z-fill rate N^2 / t_fill (entries/s) of the mixed path when its far
field is within 1e-6 of the FP64 path's, otherwise of the FP64 path; GMRES
solve seconds of both are reported beside it, and, after the timed steps,
the solve seconds at the loosest GMRES tolerance in 1e-4 .. 1e-12 whose far
field is within 1e-6 of the oracle's (dense FP64 fill and LU on the host).  The multi-RHS pass reports
its per-RHS solve time against 128 sequential single-RHS solves of the same
operator (timed once, after the timed steps).

The roofline object describes the kernel with the largest device time per
step, timed live with HIP events on the library's stream.  Its algorithmic
work per launch is derived below; the CPU baseline is the FP64 oracle's
dense fill on the host cores, followed (untimed for the baseline's value,
timed on its own) by the oracle's LU solve and far field, the reference of
every accuracy figure of the line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_VALU = 78.6      # TFLOP/s, MI355X vector FP64
PEAK_FP32_VALU = 157.3     # TFLOP/s, MI355X vector FP32
PEAK_HBM = 8000.0          # GB/s
PEAK_FP32_MFMA = 157.3     # TFLOP/s, MI355X dense FP32 matrix cores

# HBM bytes moved per launch (per fill for the regular-pair kernel: all its
# colour-class launches), from rocprofv3 FETCH_SIZE and WRITE_SIZE counters
# scaled by a 1 GiB device copy (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0).  A
# kernel changed after its counters were taken gets None here.
MEASURED_TRAFFIC = {
    ("k_regular", "fp64"): 21.77e9,    # 13.83 GB read + 7.94 GB written per fill
    ("k_regular_range", "mixed"): 3.52e9,   # 1.42 GB read + 2.10 GB written per fill
    ("k_gemv3", "fp64"): 1.291e9,
    ("k_gemv3", "mixed"): 0.683e9,
}

# Algorithmic flops of the regular-pair fill (FMA = 2 flops, every
# transcendental call = 1).  Per point pair: distance and unit vector 13,
# kernel differences 151 (two complex exponentials, f, g, phi for both
# media, D0, df, dg and the two gradient scalars), twelve weighted kernel
# values 155 -> 319.  Per element pair: trial-side contraction with the
# shape functions 7*12*6*7 complex-by-real multiply-adds (4 flops) = 14112,
# merge of a chunk's triangles by node 7*12*6 complex adds = 1008.  Per
# trial chunk of 4 triangles with ns distinct nodes: test-side contraction
# 6*12*ns*7 multiply-adds = 2016 ns.
FLOP_POINT_PAIR = 319
FLOP_PAIR_TRIAL = 14112 + 1008
FLOP_CHUNK_TEST_PER_NODE = 2016
CHUNK = 4
# Sauter-Schwab: per point two P2 evaluations with frames (2 x 310), the
# map and weights 20, kernel values 319, and the rank-one accumulation
# into the 6 x 6 x 12 block 12 * (12 + 144) -> 2831.
FLOP_SSQ_POINT = 2 * 310 + 20 + 319 + 12 * 156


def regular_fill_flops(S, tri, npairs):
    """Algorithmic flops of one regular-pair fill (all colour-class launches)
    of the solver's mesh: per element pair the point-pair work and the
    trial-side contraction, per (test triangle, trial chunk) workgroup the
    test-side contraction of its ns distinct chunk nodes."""
    nt = tri.shape[0]
    rank = np.empty_like(S.node_order)
    rank[S.node_order] = np.arange(S.nn)
    tm = rank[tri[S.tri_order]]
    ns = np.array([np.unique(tm[k:k + CHUNK]).size for k in range(0, nt, CHUNK)])
    return (npairs * (49 * FLOP_POINT_PAIR + FLOP_PAIR_TRIAL)
            + nt * int(ns.sum()) * FLOP_CHUNK_TEST_PER_NODE)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sphere1280")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--paths", default="fp64,mixed")
    ap.add_argument("--no-mrhs", action="store_true", help="skip the 128-RHS block solve pass")
    ap.add_argument("--no-grad", action="store_true", help="skip the adjoint gradient pass")
    ap.add_argument("--no-precond-study", action="store_true",
                    help="skip the preconditioner study (GMRES without vs with block-Jacobi)")
    ap.add_argument("--no-quad-study", action="store_true",
                    help="skip the comparison of the default quadrature with the paper's scheme")
    ap.add_argument("--no-spectrum-study", action="store_true",
                    help="skip the LSPR spectrum sweep of the silver spheroid")
    ap.add_argument("--no-blr-study", action="store_true",
                    help="skip the block low-rank operator beyond dense memory")
    ap.add_argument("--no-frame-study", action="store_true",
                    help="skip the comparison of the interpolated frame with node-attached tangents")
    ap.add_argument("--frame-refinement", action="store_true",
                    help="in the frame study, also run the spheroid refinement (320 / 1280 / 5120 triangles)")
    ap.add_argument("--no-tol-sweep", action="store_true",
                    help="skip the search of the loosest GMRES tolerance meeting 1e-6 far-field error")
    ap.add_argument("--no-spheroid", action="store_true",
                    help="skip the 5120-triangle plasmonic spheroid pass (FP64 and mixed, B = 256)")
    ap.add_argument("--oracle-one-core", action="store_true",
                    help="also time the oracle's full fill of the workload on one core (about 40 s)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="copy 1 GiB device to device once (scales the FETCH_SIZE / WRITE_SIZE "
                         "counters) and exit")
    ap.add_argument("--only", choices=["all", "main", "mrhs", "grad", "precond", "quad", "spectrum", "blr",
                                       "frame", "spheroid"],
                    default="all",
                    help="run one pass of the step only (for profiling); the JSON line is "
                         "printed for 'all' and 'main'")
    return ap.parse_args()


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(xyz, tri, cfg, N, khat, pol, rdirs, one_core=False):
    """The FP64 oracle on the host cores: its dense fill of the same mesh
    (timed: the baseline's value), then its dense LU solve (timed) and far
    field at the 360 cut-plane angles, the reference of the accuracy
    figures; beside it the oracle's fill of the 80-triangle sphere on all
    threads and on one, and with one_core the workload's fill on one core.
    Returns (baseline record, oracle far field)."""
    from oracle import core, galerkin
    from workloads import get_config, icosphere_p2
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    threads = max(1, min(threads, os.cpu_count() or 1))
    P = galerkin.Problem(xyz, tri, cfg["k0"], cfg["eps_r"], cfg["mu_r"])
    core.lib()
    small = {}
    c1 = get_config("sphere80")
    x1, t1 = icosphere_p2(c1["n_tris"], c1["axes"])
    P1 = galerkin.Problem(x1, t1, c1["k0"], c1["eps_r"], c1["mu_r"])
    for nth in (threads, 1):
        t0 = time.perf_counter()
        core.fill(x1, t1, P1.phys, nss=4, nthreads=nth)
        small[f"sphere80_fill_s_{nth}_threads"] = time.perf_counter() - t0
    if one_core:
        t0 = time.perf_counter()
        core.fill(xyz, tri, P.phys, nss=4, nthreads=1)
        small["fill_s_1_thread"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    K = core.fill(xyz, tri, P.phys, nss=4, nthreads=threads)
    dt = time.perf_counter() - t0
    Z = galerkin.assemble(P, *K, galerkin.mass_matrix(P))
    del K
    b = galerkin.planewave_rhs(P, khat, pol)[:, 0]
    t0 = time.perf_counter()
    x = np.linalg.solve(Z, b)
    t_lu = time.perf_counter() - t0
    del Z
    F = galerkin.far_field(P, x, rdirs)
    rec = {"value": N * N / dt, "unit": "entries/s", "cores": threads, "kind": "oracle",
           "sample": f"full FP64 dense fill (K1, K2eps, K2mu, all {tri.shape[0]}^2 element "
                     f"pairs) of the same mesh, {dt:.2f} s",
           "t_fill_s": dt, "t_lu_solve_s": t_lu, "solve": "dense LU (numpy / LAPACK zgesv)",
           "nproc": os.cpu_count(), "cpu_model": _cpu_model(), **small}
    return rec, F


TOL_LADDER = (1e-4, 1e-5, 1e-6, 1e-7, 1e-8, 1e-9, 1e-10, 1e-11, 1e-12)


def tol_sweep(S, khat, pol, rdirs, Fref, block, reps=3):
    """The solve-seconds rule of the metric: the loosest GMRES tolerance of
    the ladder whose far field is within 1e-6 of the reference, with its
    solve time (mean of reps solves from b on the device to x), iterations
    and error; every rung's error is listed."""
    S.precond_setup(block)
    b = S.rhs(khat, pol)
    rungs = []
    chosen = None
    for tol in TOL_LADDER:
        times = []
        for _ in range(reps):
            x, st, code = S.solve(b, tol=tol, maxit=800)
            times.append(st.t_solve_ms)
        F = S.farfield(x, rdirs).cpu().numpy()[0]
        err = float(np.linalg.norm(F - Fref) / np.linalg.norm(Fref))
        rungs.append({"tol": tol, "err": err, "iters": int(st.iters), "sweeps": int(st.outer_iters),
                      "t_solve_ms": float(np.mean(times)), "converged": code == 0})
        if chosen is None and code == 0 and err <= 1e-6:
            chosen = rungs[-1]
            break
    return {"rule": "loosest tol in 1e-4..1e-12 with far field within 1e-6 of the reference",
            "tol": chosen["tol"] if chosen else None,
            "solve_s": chosen["t_solve_ms"] * 1e-3 if chosen else None,
            "iters": chosen["iters"] if chosen else None,
            "err": chosen["err"] if chosen else None, "rungs": rungs}


def spheroid_pass(mbem, get_config, icosphere_p2, planewaves, rdirs, log, reps=3):
    """The 5120-triangle plasmonic spheroid (40968 unknowns, k_a = 4,
    eps_r = -10 + 1i, block-Jacobi B = 256, one plane wave): FP64, mixed with
    the FP64 near store (the workload's complex64 storage with FP64
    near-field blocks) and mixed without it; fill and solve to 1e-6
    (iterations, times), every far field against an FP64 solve to 1e-10."""
    c = get_config("spheroid5120")
    xyz, tri = icosphere_p2(c["n_tris"], c["axes"])
    kh, po = planewaves("spheroid5120")
    out = {"workload": "spheroid5120", "n_tris": int(tri.shape[0]), "unknowns": 4 * int(xyz.shape[0]),
           "k0": c["k0"], "eps_r": str(c["eps_r"]), "mbj_block": c["mbj_block"], "gmres_tol": c["tol"]}
    F = {}
    for name, prec, store in (("fp64", mbem.MBEM_FP64, False), ("mixed", mbem.MBEM_MIXED, True),
                              ("mixed_no_store", mbem.MBEM_MIXED, False)):
        S = mbem.Solver(xyz, tri, c["k0"], c["eps_r"], c["mu_r"], precision=prec, near_store=store)
        try:
            fs = [S.fill() for _ in range(reps)]
            ps = S.precond_setup(c["mbj_block"])
            b = S.rhs(kh, po)
            sols = [S.solve(b, tol=c["tol"], maxit=1000) for _ in range(reps)]
            x, st, code = sols[-1]
            Fp = S.farfield(x, rdirs).cpu().numpy()[0]
            rec = {"t_fill_ms": float(np.mean([f.t_fill_ms for f in fs])),
                   "t_regular_ms": float(np.mean([f.t_regular_ms for f in fs])),
                   "t_near_ms": float(np.mean([f.t_near_ms for f in fs])),
                   "t_singular_ms": float(np.mean([f.t_ssq_ms for f in fs])),
                   "fill_rate": (4 * xyz.shape[0]) ** 2 / (1e-3 * float(np.mean([f.t_fill_ms for f in fs]))),
                   "t_setup_ms": ps.t_setup_ms,
                   "t_solve_ms": float(np.mean([s[1].t_solve_ms for s in sols])),
                   "iters": int(st.iters), "sweeps": int(st.outer_iters), "rel_resid": float(st.rel_resid),
                   "converged": code == 0, "n_near_pairs": int(fs[-1].n_near_pairs), "near_store": store}
            xt, stt, codet = S.solve(b, tol=1e-10, maxit=1000)
            F[name + "@1e-10"] = S.farfield(xt, rdirs).cpu().numpy()[0]
            rec["iters_at_1e-10"] = int(stt.iters)
            F[name] = Fp
            out[name] = rec
            log(f"spheroid5120 {name}: fill {rec['t_fill_ms']:.1f} ms, solve {rec['t_solve_ms']:.1f} ms, "
                f"{rec['iters']} iterations")
        finally:
            S.close()
    rel = lambda a, b: float(np.linalg.norm(F[a] - F[b]) / np.linalg.norm(F[b]))
    ref = "fp64@1e-10"
    out["farfield_err_vs_fp64_at_1e-10"] = {k: rel(k, ref) for k in F if k != ref}
    return out


PRECOND_STUDY = (("sphere1280", (50, 100, 256, 512), 1500),
                 ("spheroid5120", (50, 100, 256, 512), 2000),
                 ("spheroid_lspr@506nm", (50, 100, 256, 512), 2000))
PRECOND_TOL = 1e-5        # the tolerance of the paper's preconditioner comparisons


def _precond_case(name, get_config, icosphere_p2, planewaves):
    """(xyz, tri, k0, eps_r, mu_r, khat, pol) of a preconditioner-study case."""
    if name == "spheroid_lspr@506nm":
        from workloads import spectrum_workload
        xyz, tri, _, k0, eps, kh, po, _ = spectrum_workload("spheroid_lspr", [506.0])
        return xyz, tri, float(k0[0]), complex(eps[0]), 1.0, kh[None], po[None]
    c = get_config(name)
    xyz, tri = icosphere_p2(c["n_tris"], c["axes"])
    kh, po = planewaves(name)
    return xyz, tri, c["k0"], c["eps_r"], c["mu_r"], kh, po


def precond_study(mbem, get_config, icosphere_p2, planewaves, log):
    """GMRES iterations and times without a preconditioner and with Morton
    block-Jacobi over a sweep of the cluster size, FP64 operator, one plane
    wave, tolerance 1e-5; run once after the timed steps."""
    out = {}
    for wl, blocks, maxit in PRECOND_STUDY:
        xyz, tri, k0, eps, mu, kh, po = _precond_case(wl, get_config, icosphere_p2, planewaves)
        S = mbem.Solver(xyz, tri, k0, eps, mu, precision=mbem.MBEM_FP64)
        try:
            fs = S.fill()
            b = S.rhs(kh, po)
            n2 = S.N // 2
            res = {"unknowns": S.N, "k0": k0, "eps_r": str(eps), "tol": PRECOND_TOL,
                   "precision": "fp64", "t_fill_ms": fs.t_fill_ms}
            S.precond_setup(0)
            x, st, code = S.solve(b, tol=PRECOND_TOL, maxit=maxit)
            base = {"iters": st.iters, "t_solve_ms": st.t_solve_ms, "converged": code == 0,
                    "rel_resid": st.rel_resid}
            res["none"] = base
            log(f"precond study {wl}: no preconditioner {st.iters} iterations")
            for B in blocks:
                ps = S.precond_setup(B)
                x, st, code = S.solve(b, tol=PRECOND_TOL, maxit=maxit)
                nb = (n2 + B - 1) // B
                res[f"B{B}"] = {"blocks": nb, "mbytes": nb * (2 * B) ** 2 * 16 / 1e6,
                                "t_setup_ms": ps.t_setup_ms, "iters": st.iters,
                                "t_solve_ms": st.t_solve_ms, "converged": code == 0,
                                "rel_resid": st.rel_resid,
                                "iter_reduction": base["iters"] / max(1, st.iters),
                                "solve_speedup": base["t_solve_ms"] / max(1e-9, st.t_solve_ms)}
                log(f"precond study {wl}: B = {B}, {st.iters} iterations")
            out[wl] = res
        finally:
            S.close()
    return out


def spectrum_study(mbem, log):
    """The LSPR spectrum of the silver spheroid in one sweep call per
    precision (the first point includes the one geometry build)."""
    from workloads import spectrum_workload
    xyz, tri, lam, k0, eps, kh, po, c = spectrum_workload("spheroid_lspr")
    out = {"workload": "spheroid_lspr", "n_tris": int(tri.shape[0]), "n_nodes": int(xyz.shape[0]),
           "unknowns": 4 * int(xyz.shape[0]), "points": int(lam.shape[0]),
           "lambda_nm": [float(lam[0]), float(lam[-1])], "mbj_block": c["mbj_block"],
           "tol": c["tol"]}
    sig = {}
    npts = lam.shape[0]
    for name, prec in (("fp64", mbem.MBEM_FP64), ("mixed", mbem.MBEM_MIXED)):
        S = mbem.Solver(xyz, tri, 1.0, 1.0, precision=prec)
        try:
            t0 = time.perf_counter()
            # mixed: one inner GMRES to the sweep's tolerance, then the FP64
            # residual check
            sg, it, st = S.spectrum(k0, eps, kh, po, block=c["mbj_block"], tol=c["tol"],
                                    maxit=800, inner_tol=c["tol"])
            wall = time.perf_counter() - t0
            flops = regular_fill_flops(S, tri, st.n_regular_pairs)
        finally:
            S.close()
        sig[name] = sg
        i = int(np.argmax(sg[:, 0]))
        t_reg = st.t_regular_ms / npts
        gemv_ms = st.t_matvec_ms / max(1, st.n_matvec)
        n2 = 2 * xyz.shape[0]
        gemv_bytes = 3 * n2 * n2 * (16 if name == "fp64" else 8) + 4 * n2 * 16
        peak = PEAK_FP64_VALU
        out[name] = {"wall_s": wall, "points_per_s": npts / wall,
                     # FP64: every regular pair in FP64; mixed: the FP32 kernel, which
                     # evaluates its near pairs in FP64 (on this electrically small,
                     # high-contrast body most pairs are near)
                     "k_regular": ({"ms_per_point": t_reg, "tflops": flops / (t_reg * 1e-3) / 1e12,
                                    "peak": peak, "frac": flops / (t_reg * 1e-3) / 1e12 / peak}
                                   if name == "fp64" else
                                   {"ms_per_point": t_reg,
                                    "near_pair_fraction": st.n_near_pairs / npts / max(1, st.n_regular_pairs)}),
                     "k_gemv3": {"ms_per_launch": gemv_ms,
                                 "gbps": gemv_bytes / (gemv_ms * 1e-3) / 1e9,
                                 "frac": gemv_bytes / (gemv_ms * 1e-3) / 1e9 / PEAK_HBM},
                     "t_fill_ms": st.t_fill_ms, "t_setup_ms": st.t_setup_ms,
                     "t_solve_ms": st.t_solve_ms,
                     "iters_total": int(st.iters), "iters_max": int(it.max()),
                     "worst_rel_resid": st.rel_resid,
                     "peak_lambda_nm": float(lam[i]), "peak_c_ext_nm2": float(sg[i, 0]),
                     "energy_balance_max": float(np.abs((sg[:, 1] + sg[:, 2]) / sg[:, 0] - 1).max())}
        log(f"spectrum study {name}: {lam.shape[0]} points in {wall:.2f} s, peak "
            f"{sg[i, 0]:.0f} nm^2 at {lam[i]:.0f} nm")
    out["mixed_vs_fp64_max_rel"] = float(np.abs(sig["mixed"] / sig["fp64"] - 1).max())
    return out


BLR_STUDY = dict(n_tris=20480, k0=5.0, eps_r=2.25,
                 opts=dict(cluster=512, eta=2.0, eps=1e-6, rmax=128), block=100, tol=1e-8)


def blr_study(mbem, icosphere_p2, log):
    """Block low-rank operator beyond dense memory (see the module docstring);
    its accuracy against the Mie series is checked by the GPU tests, here the
    energy balance C_ext = C_sca + C_abs (a lossless sphere) is reported."""
    c = BLR_STUDY
    xyz, tri = icosphere_p2(c["n_tris"])
    S = mbem.Solver(xyz, tri, c["k0"], c["eps_r"])
    try:
        bs = S.fill_compressed(**c["opts"])
        ps = S.precond_setup(c["block"])
        kh, po = np.array([0, 0, 1.0]), np.array([1.0, 0, 0], dtype=np.complex128)
        x, st, code = S.solve(S.rhs(kh, po), c["tol"], maxit=800)
        cs = S.cross_sections(x[0], kh, po)
        mv = st.t_matvec_ms / max(1, st.n_matvec)
        # bytes of one product: every stored tile once, x twice per block, t out
        mv_bytes = bs.stored_bytes + 4 * S.N * 16
        out = {"workload": f"sphere{c['n_tris']}", "unknowns": S.N, "k0": c["k0"], "eps_r": c["eps_r"],
               "options": c["opts"], "t_fill_ms": bs.t_total_ms, "t_band_fill_ms": bs.t_fill_ms,
               "t_aca_ms": bs.t_aca_ms, "stored_gb": bs.stored_bytes / 1e9,
               "dense_gb": bs.dense_bytes / 1e9, "stored_fraction": bs.stored_bytes / bs.dense_bytes,
               "clusters": bs.n_clusters, "lowrank_tiles": bs.n_lowrank, "tiles": bs.n_tiles,
               "mean_rank": bs.mean_rank, "max_rank": bs.max_rank,
               "matvec_ms": mv, "matvec_gbps": mv_bytes / (mv * 1e-3) / 1e9,
               "matvec_hbm_frac": mv_bytes / (mv * 1e-3) / 1e9 / PEAK_HBM,
               "t_setup_ms": ps.t_setup_ms if ps is not None else None,
               "gmres_iters": st.iters, "t_solve_ms": st.t_solve_ms, "converged": code == 0,
               "c_ext": cs[0], "c_sca": cs[1], "c_abs": cs[2]}
        out["energy_balance"] = (cs[1] + cs[2]) / cs[0] - 1
        log(f"compressed study: {S.N} unknowns, {bs.stored_bytes / 1e9:.1f} of {bs.dense_bytes / 1e9:.1f} GB, "
            f"fill {bs.t_total_ms:.0f} ms, product {mv:.2f} ms, {st.iters} iterations")
        return out
    finally:
        S.close()


def frame_study(mbem, get_config, icosphere_p2, planewaves, rdirs, log, reps=3, refinement=True):
    """The interpolated frame (the paper's construction, the default) against
    node-attached tangents on the 1280-triangle sphere, FP64 and mixed: fill
    times, GMRES iterations to 1e-8, the energy balance
    |C_ext - C_sca - C_abs| / C_ext of each solution (the sphere is lossless,
    so the gap is discretisation error), and the far-field difference of the
    two bases."""
    c = get_config("sphere1280")
    xyz, tri = icosphere_p2(c["n_tris"], c["axes"])
    kh, po = planewaves("sphere1280")
    out = {"workload": "sphere1280", "unknowns": None}
    F = {}
    for name, prec, frame in (("interpolated_fp64", mbem.MBEM_FP64, mbem.MBEM_FRAME_INTERPOLATED),
                              ("nodal_fp64", mbem.MBEM_FP64, mbem.MBEM_FRAME_NODAL),
                              ("interpolated_mixed", mbem.MBEM_MIXED, mbem.MBEM_FRAME_INTERPOLATED),
                              ("nodal_mixed", mbem.MBEM_MIXED, mbem.MBEM_FRAME_NODAL)):
        S = mbem.Solver(xyz, tri, c["k0"], c["eps_r"], c["mu_r"], precision=prec, frame=frame)
        try:
            fs = [S.fill() for _ in range(reps + 1)][1:]
            S.precond_setup(c["mbj_block"])
            x, st, code = S.solve(S.rhs(kh, po), tol=c["tol"], maxit=600)
            F[name] = S.farfield(x, rdirs).cpu().numpy()[0]
            cs = S.cross_sections(x[0], kh[0], po[0])
            out["unknowns"] = S.N
            out[name] = {"t_fill_ms": float(np.mean([f.t_fill_ms for f in fs])),
                         "t_regular_ms": float(np.mean([f.t_regular_ms for f in fs])),
                         "t_singular_ms": float(np.mean([f.t_ssq_ms for f in fs])),
                         "iters": st.iters, "converged": code == 0,
                         "c_ext": float(cs[0]),
                         "energy_balance": float(abs(cs[0] - cs[1] - cs[2]) / cs[0])}
            log(f"frame study: {name} fill {out[name]['t_fill_ms']:.2f} ms, "
                f"energy balance {out[name]['energy_balance']:.2e}")
        finally:
            S.close()
    rel = lambda a, b: float(np.linalg.norm(F[a] - F[b]) / np.linalg.norm(F[b]))
    out["farfield_nodal_vs_interpolated_fp64"] = rel("nodal_fp64", "interpolated_fp64")
    out["farfield_nodal_mixed_vs_nodal_fp64"] = rel("nodal_mixed", "nodal_fp64")
    out["spheroid_refinement"] = frame_refinement(mbem, get_config, icosphere_p2, log) if refinement else None
    return out


def frame_refinement(mbem, get_config, icosphere_p2, log):
    """Both bases under refinement on the plasmonic spheroid of the
    spheroid5120 workload (semi-axes 1, 1, 2, eps_r = -10 + 1i, k_a = 4),
    oblique incidence (45 degrees to the axis), 320 / 1280 / 5120 triangles,
    FP64, GMRES to 1e-10: C_ext, C_abs and the energy balance per mesh.
    There is no closed form for a spheroid; the change of C_ext between
    consecutive meshes measures the convergence."""
    c = get_config("spheroid5120")
    kh = np.array([np.sqrt(0.5), 0.0, np.sqrt(0.5)])
    po = np.array([np.sqrt(0.5), 0.0, -np.sqrt(0.5)], dtype=np.complex128)
    out = {}
    for name, frame in (("interpolated", mbem.MBEM_FRAME_INTERPOLATED), ("nodal", mbem.MBEM_FRAME_NODAL)):
        rows = []
        for nt in (320, 1280, 5120):
            xyz, tri = icosphere_p2(nt, c["axes"])
            S = mbem.Solver(xyz, tri, c["k0"], c["eps_r"], c["mu_r"], frame=frame)
            try:
                S.fill()
                S.precond_setup(c["mbj_block"])
                x, st, code = S.solve(S.rhs(kh[None], po[None]), tol=1e-10, maxit=800)
                cs = S.cross_sections(x[0], kh, po)
                rows.append({"n_tris": nt, "c_ext": float(cs[0]), "c_sca": float(cs[1]), "c_abs": float(cs[2]),
                             "energy_balance": float(abs(cs[0] - cs[1] - cs[2]) / cs[0]), "iters": st.iters,
                             "converged": code == 0})
            finally:
                S.close()
            log(f"frame refinement: {name} {nt} C_ext {rows[-1]['c_ext']:.6f} "
                f"balance {rows[-1]['energy_balance']:.1e}")
        out[name] = rows
    return out


def quad_study(mbem, get_config, icosphere_p2, planewaves, rdirs, log, reps=3):
    """The paper's own quadrature (12-point rule, Sauter-Schwab on the
    singular kernels, 12-point remainder) against the default on the
    1280-triangle sphere: fill times and the far-field difference of the two
    (FP64 and mixed), GMRES to 1e-8."""
    c = get_config("sphere1280")
    xyz, tri = icosphere_p2(c["n_tris"], c["axes"])
    kh, po = planewaves("sphere1280")
    out = {"workload": "sphere1280", "unknowns": None}
    F = {}
    for name, prec, quad in (("default_fp64", mbem.MBEM_FP64, mbem.MBEM_QUAD_DEFAULT),
                             ("paper_fp64", mbem.MBEM_FP64, mbem.MBEM_QUAD_PAPER),
                             ("default_mixed", mbem.MBEM_MIXED, mbem.MBEM_QUAD_DEFAULT),
                             ("paper_mixed", mbem.MBEM_MIXED, mbem.MBEM_QUAD_PAPER)):
        S = mbem.Solver(xyz, tri, c["k0"], c["eps_r"], c["mu_r"], precision=prec, quadrature=quad)
        try:
            fs = [S.fill() for _ in range(reps + 1)][1:]
            S.precond_setup(c["mbj_block"])
            x, st, code = S.solve(S.rhs(kh, po), tol=c["tol"], maxit=600)
            F[name] = S.farfield(x, rdirs).cpu().numpy()[0]
            out["unknowns"] = S.N
            out[name] = {"t_fill_ms": float(np.mean([f.t_fill_ms for f in fs])),
                         "t_regular_ms": float(np.mean([f.t_regular_ms for f in fs])),
                         "t_singular_ms": float(np.mean([f.t_ssq_ms for f in fs])),
                         "fill_rate": S.N ** 2 / (1e-3 * float(np.mean([f.t_fill_ms for f in fs]))),
                         "iters": st.iters, "converged": code == 0}
            log(f"quadrature study: {name} fill {out[name]['t_fill_ms']:.2f} ms")
        finally:
            S.close()
    rel = lambda a, b: float(np.linalg.norm(F[a] - F[b]) / np.linalg.norm(F[b]))
    out["farfield_paper_vs_default_fp64"] = rel("paper_fp64", "default_fp64")
    out["farfield_paper_mixed_vs_paper_fp64"] = rel("paper_mixed", "paper_fp64")
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the method "
              "is benchmarked on a single MI355X", file=sys.stderr)
        sys.exit(2)
    import torch
    if args.copy_calibration:
        a = torch.ones(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 1 << 30}), flush=True)
        return
    from paper_2604_21181_amd import mbem
    from workloads import get_config, icosphere_p2, planewaves
    from workloads.configs import cut_plane_directions

    if args.only != "all":
        # one pass of the step, or one study
        keep = {"mrhs": "no_mrhs", "grad": "no_grad", "precond": "no_precond_study",
                "quad": "no_quad_study", "spectrum": "no_spectrum_study", "blr": "no_blr_study",
                "frame": "no_frame_study", "spheroid": "no_spheroid"}
        for name, flag in keep.items():
            if name != args.only:
                setattr(args, flag, True)
        if args.only != "main":
            args.paths = ""
            args.no_cpu_baseline = True
            args.no_tol_sweep = True
        if args.only in ("precond", "quad", "spectrum", "blr", "frame", "spheroid"):
            args.steps, args.warmup = 0, 0
    cfg = get_config(args.workload)
    xyz, tri = icosphere_p2(cfg["n_tris"], cfg["axes"])
    khat, pol = planewaves(args.workload)
    rdirs = cut_plane_directions(360)
    paths = [p for p in args.paths.split(",") if p]
    prec = {"fp64": mbem.MBEM_FP64, "mixed": mbem.MBEM_MIXED}
    solvers = {p: mbem.Solver(xyz, tri, cfg["k0"], cfg["eps_r"], cfg["mu_r"], precision=prec[p])
               for p in paths}
    N = solvers[paths[0]].N if paths else 0
    nt = tri.shape[0]
    Smr = None
    if not args.no_mrhs:
        mcfg = get_config("sphere1280_mrhs")
        mxyz, mtri = icosphere_p2(mcfg["n_tris"], mcfg["axes"])
        mkh, mpol = planewaves("sphere1280_mrhs")
        Smr = mbem.Solver(mxyz, mtri, mcfg["k0"], mcfg["eps_r"], mcfg["mu_r"],
                          precision=mbem.MBEM_MIXED)
    Sg = None
    if not args.no_grad:
        gcfg = get_config("ellipsoid1280")
        gxyz, gtri = icosphere_p2(gcfg["n_tris"], gcfg["axes"])
        gkh, gpol = planewaves("ellipsoid1280")
        Sg = mbem.Solver(gxyz, gtri, gcfg["k0"], gcfg["eps_r"], gcfg["mu_r"], precision=mbem.MBEM_FP64)

    def step():
        out = {}
        for p in paths:
            S = solvers[p]
            fs = S.fill()
            ps = S.precond_setup(cfg["mbj_block"])
            b = S.rhs(khat, pol)
            x, ss, code = S.solve(b, tol=cfg["tol"], maxit=600)
            F = S.farfield(x, rdirs)
            out[p] = dict(fill=fs.as_dict(), setup_ms=ps.t_setup_ms, solve=ss.as_dict(), code=code,
                          F=F, x=x)
        if Smr is not None:
            fs = Smr.fill()
            ps = Smr.precond_setup(mcfg["mbj_block"])
            b = Smr.rhs(mkh, mpol)
            x, bs, code = Smr.solve_block(b, mcfg["tol"])
            F = Smr.farfield(x, mkh)              # every solution in every incidence direction
            out["mrhs"] = dict(fill=fs.as_dict(), setup_ms=ps.t_setup_ms, solve=bs.as_dict(),
                               code=code, F=F, b=b)
        if Sg is not None:
            t0 = time.perf_counter()
            fs = Sg.fill()
            ps = Sg.precond_setup(gcfg["mbj_block"])
            b = Sg.rhs(gkh, gpol)
            x, ss, code = Sg.solve(b, tol=gcfg["tol"], maxit=600)
            g, ags, lam, dnode, dx = Sg.grad_sigma_ext(x[0], gkh[0], gpol[0], tol=gcfg["tol"], shape=True)
            torch.cuda.synchronize()
            out["grad"] = dict(fill=fs.as_dict(), setup_ms=ps.t_setup_ms, solve=ss.as_dict(), code=code,
                               adj=ags.as_dict(), out=g, dnode_norm=float(torch.linalg.norm(dnode)),
                               wall_ms=1e3 * (time.perf_counter() - t0))
        return out

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    log(f"{args.workload}: {nt} triangles, N = {N}, paths {paths}")
    for i in range(args.warmup):
        step()
        log(f"warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    recs = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        recs.append(step())
        log(f"step {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1e3 * wall / max(1, args.steps)

    def mean(path, sect, key):
        return float(np.mean([r[path][sect][key] for r in recs]))

    if paths:
        res = {}
        for p in paths:
            res[p] = dict(
                t_fill_ms=mean(p, "fill", "t_fill_ms"),
                t_regular_ms=mean(p, "fill", "t_regular_ms"),
                t_near_ms=mean(p, "fill", "t_near_ms"),
                t_ssq_ms=mean(p, "fill", "t_ssq_ms"),
                t_geom_ms=mean(p, "fill", "t_geom_ms"),
                t_mass_ms=mean(p, "fill", "t_mass_ms"),
                t_setup_ms=float(np.mean([r[p]["setup_ms"] for r in recs])),
                t_solve_ms=mean(p, "solve", "t_solve_ms"),
                t_matvec_ms=mean(p, "solve", "t_matvec_ms"),
                n_matvec=int(recs[-1][p]["solve"]["n_matvec"]),
                iters=int(recs[-1][p]["solve"]["iters"]),
                outer=int(recs[-1][p]["solve"]["outer_iters"]),
                rel_resid=float(recs[-1][p]["solve"]["rel_resid"]),
                n_near=int(recs[-1][p]["fill"]["n_near_pairs"]),
                n_regular=int(recs[-1][p]["fill"]["n_regular_pairs"]),
            )
            res[p]["fill_rate"] = N * N / (res[p]["t_fill_ms"] * 1e-3)

        last = recs[-1]
        ff = {p: last[p]["F"].cpu().numpy()[0] for p in paths}
        info = {}
        mixed_ok = False
        if "fp64" in paths and "mixed" in paths:
            e = float(np.linalg.norm(ff["mixed"] - ff["fp64"]) / np.linalg.norm(ff["fp64"]))
            info["farfield_err_mixed_vs_fp64"] = e
            mixed_ok = e <= 1e-6
        head = "mixed" if (mixed_ok or paths == ["mixed"]) else paths[0]

        # ---- rooflines of the candidate kernels; `roofline` is the one with
        # the largest device time per step
        def roofline_of(kname, kp):
            r = res[kp]
            n2 = N // 2
            if kname == "gemv":
                esz = 16 if kp == "fp64" else 8
                traffic = 3 * n2 * n2 * esz + 2 * N * 16            # three blocks + x in, y out
                per_launch_ms = r["t_matvec_ms"] / max(1, r["n_matvec"])
                achieved = traffic / (per_launch_ms * 1e-3) / 1e9
                return {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM, "unit": "GB/s",
                        "frac": achieved / PEAK_HBM, "traffic": MEASURED_TRAFFIC.get(("k_gemv3", kp)),
                        "kernel": "k_gemv3", "path": kp,
                        "algorithmic_bytes_per_launch": traffic, "launch_ms": per_launch_ms}
            if kname == "regular":
                flops = regular_fill_flops(solvers[kp], tri, r["n_regular"])
                achieved = flops / (r["t_regular_ms"] * 1e-3) / 1e12
                peak = PEAK_FP64_VALU if kp == "fp64" else PEAK_FP32_VALU
                kern = "k_regular" if kp == "fp64" else "k_regular_range"
                return {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                        "frac": achieved / peak, "traffic": MEASURED_TRAFFIC.get((kern, kp)),
                        "kernel": kern, "path": kp,
                        "algorithmic_flops_per_launch": flops, "launch_ms": r["t_regular_ms"]}
            S = solvers[kp]
            ncoinc, nedge, nvert = S.n_singular
            pts = (6 * ncoinc + 5 * nedge + 2 * nvert) * 256
            flops = pts * FLOP_SSQ_POINT
            achieved = flops / (r["t_ssq_ms"] * 1e-3) / 1e12
            return {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_VALU, "unit": "TFLOP/s",
                    "frac": achieved / PEAK_FP64_VALU, "traffic": None, "kernel": "k_ssq", "path": kp,
                    "algorithmic_flops_per_launch": flops, "launch_ms": r["t_ssq_ms"]}

        cand = []
        for p in paths:
            r = res[p]
            cand.append((r["t_regular_ms"], "regular", p))
            cand.append((r["t_ssq_ms"], "ssq", p))
            if r["n_matvec"]:
                # the solve times a sample of its products: scale to all of them
                cand.append((r["t_matvec_ms"] / r["n_matvec"] * r["iters"], "gemv", p))
        cand.sort(reverse=True)
        rooflines = [roofline_of(kname, kp) for _, kname, kp in cand]
        roof = dict(rooflines[0])
        roof.pop("path", None)

    cpu, Foracle = None, None
    if paths and not args.no_cpu_baseline:
        log("timing the CPU oracle (dense fill, LU solve, far field)")
        cpu, Foracle = cpu_baseline(xyz, tri, cfg, N, khat, pol, rdirs, one_core=args.oracle_one_core)
        for p in paths:
            info[f"farfield_err_{p}_vs_oracle"] = float(np.linalg.norm(ff[p] - Foracle) / np.linalg.norm(Foracle))
    sweeps = None
    if paths and not args.no_tol_sweep:
        # reference: the oracle's LU far field, else the FP64 path at 1e-12
        Fref, ref_name = Foracle, "oracle dense LU"
        if Fref is None:
            S = solvers.get("fp64") or solvers[paths[0]]
            S.precond_setup(cfg["mbj_block"])
            xr, _, _ = S.solve(S.rhs(khat, pol), tol=1e-12, maxit=800)
            Fref, ref_name = S.farfield(xr, rdirs).cpu().numpy()[0], "GPU FP64 path at tol 1e-12"
        sweeps = {"reference": ref_name}
        for p in paths:
            sweeps[p] = tol_sweep(solvers[p], khat, pol, rdirs, Fref, cfg["mbj_block"])
            log(f"tolerance sweep {p}: tol {sweeps[p]['tol']}, solve {sweeps[p]['solve_s']} s")

    mrhs = None
    if Smr is not None:
        mr = recs[-1]["mrhs"]
        bsd = [r["mrhs"]["solve"] for r in recs]
        t_block = float(np.mean([d["t_solve_ms"] for d in bsd]))
        n_gemm = sum(d["n_gemm"] for d in bsd)
        t_gemm = sum(d["t_gemm_ms"] for d in bsd) / max(1, n_gemm)
        nr = mkh.shape[0]
        mn2 = Smr.N // 2
        gflop = 32.0 * nr * mn2 * mn2                     # K1 on 2 nr, K2 on nr + nr columns
        # C_ext of every right-hand side by the optical theorem: a sphere's
        # is the same for every incidence, up to the mesh's anisotropy
        F = mr["F"].cpu().numpy()
        cext = np.array([4 * np.pi / mcfg["k0"] * np.imag(np.vdot(mpol[r], F[r, r])) for r in range(nr)])
        log("timing 128 sequential single-RHS solves of the same operator")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its = 0
        for c in range(nr):
            xs, ss, code = Smr.solve(mr["b"][c], tol=mcfg["tol"], maxit=600)
            its += ss.iters
        torch.cuda.synchronize()
        t_seq = 1e3 * (time.perf_counter() - t0)
        mrhs = {
            "workload": "sphere1280_mrhs", "nrhs": nr, "unknowns": Smr.N, "k0": mcfg["k0"],
            "eps_r": str(mcfg["eps_r"]), "gmres_tol": mcfg["tol"],
            "t_fill_ms": float(np.mean([r["mrhs"]["fill"]["t_fill_ms"] for r in recs])),
            "t_setup_ms": float(np.mean([r["mrhs"]["setup_ms"] for r in recs])),
            "t_block_solve_ms": t_block, "block_iters": int(bsd[-1]["iters"]),
            "sweeps": int(bsd[-1]["sweeps"]), "block": int(bsd[-1]["block"]),
            "gemm_config": int(bsd[-1]["gemm_config"]), "rel_resid": float(bsd[-1]["rel_resid"]),
            "ms_per_rhs_block": t_block / nr, "ms_per_rhs_sequential": t_seq / nr,
            "sequential_iters": its, "speedup_vs_sequential": t_seq / t_block,
            "cext_mean": float(cext.mean()),
            "cext_rel_spread": float((cext.max() - cext.min()) / cext.mean()),
            "gemm": {"bound": "mfma", "achieved": gflop / (t_gemm * 1e-3) / 1e12,
                     "peak": PEAK_FP32_MFMA, "unit": "TFLOP/s",
                     "frac": gflop / (t_gemm * 1e-3) / 1e12 / PEAK_FP32_MFMA,
                     "kernel": "k_cgemm_f32", "algorithmic_flops_per_launch": gflop,
                     "launch_ms": t_gemm},
        }

    grad = None
    if Sg is not None:
        gr = [r["grad"] for r in recs]
        gm = lambda f: float(np.mean([f(r) for r in gr]))
        grad = {
            "workload": "ellipsoid1280", "unknowns": Sg.N, "n_nodes": Sg.nn, "k0": gcfg["k0"],
            "eps_r": str(gcfg["eps_r"]), "gmres_tol": gcfg["tol"],
            "sigma_ext": float(gr[-1]["out"][0]),
            "dsigma_deps_re": float(gr[-1]["out"][1]), "dsigma_deps_im": float(gr[-1]["out"][2]),
            "dsigma_dnode_norm": gr[-1]["dnode_norm"],
            "t_fill_ms": gm(lambda r: r["fill"]["t_fill_ms"]),
            "t_setup_ms": gm(lambda r: r["setup_ms"]),
            "t_solve_ms": gm(lambda r: r["solve"]["t_solve_ms"]),
            "t_adjoint_solve_ms": gm(lambda r: r["adj"]["t_adjoint_ms"]),
            "t_deps_ms": gm(lambda r: r["adj"]["t_deps_ms"]),
            "t_shape_ms": gm(lambda r: r["adj"]["t_shape_ms"]),
            "t_pass_ms": gm(lambda r: r["wall_ms"]),
            "adjoint_iters": int(gr[-1]["adj"]["iters"]),
        }

    pstudy = None
    if not args.no_precond_study:
        pstudy = precond_study(mbem, get_config, icosphere_p2, planewaves, log)
    qstudy = None
    if not args.no_quad_study:
        qstudy = quad_study(mbem, get_config, icosphere_p2, planewaves, rdirs, log)
    sstudy = None
    if not args.no_spectrum_study:
        sstudy = spectrum_study(mbem, log)
    bstudy = None
    if not args.no_blr_study:
        bstudy = blr_study(mbem, icosphere_p2, log)
    spheroid = None
    if not args.no_spheroid:
        spheroid = spheroid_pass(mbem, get_config, icosphere_p2, planewaves, rdirs, log)
    fstudy = None
    if not args.no_frame_study:
        fstudy = frame_study(mbem, get_config, icosphere_p2, planewaves, rdirs, log,
                             refinement=args.frame_refinement)

    if not paths:
        # profiling run of one pass: its own section only
        print(json.dumps({"pass": args.only, "steps": args.steps, "warmup": args.warmup,
                          "ms_per_step": ms_per_step, "multi_rhs": mrhs, "gradient": grad,
                          "precond_study": pstudy, "quadrature_study": qstudy,
                          "spectrum_study": sstudy, "blr_study": bstudy, "frame_study": fstudy,
                          "spheroid5120": spheroid}),
              flush=True)
        for S in (Smr, Sg):
            if S is not None:
                S.close()
        return

    line = {
        "metric": "Z fill (entries/s) + GMRES solve s at 1e-6 far-field err; mixed vs FP64",
        "value": res[head]["fill_rate"],
        "unit": "entries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64/f32+f64" if head == "mixed" else "c128/f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n_tris": nt, "n_nodes": int(xyz.shape[0]),
                   "unknowns": N, "k0": cfg["k0"], "eps_r": str(cfg["eps_r"]),
                   "headline_path": head, "gmres_tol": cfg["tol"], "mbj_block": cfg["mbj_block"]},
        "paths": {p: {k: v for k, v in res[p].items()} for p in paths},
        "solve_s": {p: res[p]["t_solve_ms"] * 1e-3 for p in paths},
        "solve_s_at_1e-6_farfield": ({p: sweeps[p]["solve_s"] for p in paths} if sweeps else None),
        "tol_sweep": sweeps,
        "accuracy": info,
        "roofline": roof,
        "rooflines": rooflines,
        "multi_rhs": mrhs,
        "gradient": grad,
        "precond_study": pstudy,
        "quadrature_study": qstudy,
        "spectrum_study": sstudy,
        "blr_study": bstudy,
        "frame_study": fstudy,
        "spheroid5120": spheroid,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    for S in solvers.values():
        S.close()
    if Smr is not None:
        Smr.close()
    if Sg is not None:
        Sg.close()


if __name__ == "__main__":
    main()
