"""The five synthetic workloads and their seeded incidence sets.

Lengths are in units of the sphere radius; vacuum exterior (eps_a = mu_a = 1),
so the exterior wavenumber k_a equals the angular frequency.

  sphere80     unit sphere, 80 P2 triangles (162 nodes, 648 unknowns),
               k_a = 1, eps_r = 4; one x-polarised wave along +z.
  sphere1280   unit sphere, 1280 triangles (2562 nodes, 10248 unknowns),
               k_a = 5, eps_r = 2.25; FP64 vs mixed path, 360 far-field angles.
  spheroid5120 spheroid semi-axes (1,1,2), 5120 triangles (10242 nodes,
               40968 unknowns), k_a = 4, eps_r = -10 + 1i; block size 256;
               complex64 storage with FP64 near-field blocks (the near store).
  sphere1280_mrhs  the 1280-triangle sphere at k_a = 3, eps_r = 6 with 128
               right-hand sides (64 seeded directions x 2 polarisations).
  ellipsoid1280  ellipsoid semi-axes (1, 0.8, 0.6), 1280 triangles,
               k_a = 3, eps_r = 3 + 0.1i; gradient workload.

Node counts follow the closed-surface rule n_nodes = 2 F + 2.
"""
from __future__ import annotations

import numpy as np

CONFIGS = {
    "sphere80": dict(n_tris=80, axes=(1.0, 1.0, 1.0), k0=1.0, eps_r=4.0 + 0j,
                     mu_r=1.0 + 0j, mbj_block=100, tol=1e-10, nrhs=1),
    "sphere1280": dict(n_tris=1280, axes=(1.0, 1.0, 1.0), k0=5.0,
                       eps_r=2.25 + 0j, mu_r=1.0 + 0j, mbj_block=100,
                       tol=1e-8, nrhs=1),
    "spheroid5120": dict(n_tris=5120, axes=(1.0, 1.0, 2.0), k0=4.0,
                         eps_r=-10.0 + 1.0j, mu_r=1.0 + 0j, mbj_block=256,
                         tol=1e-6, nrhs=1, near_store=True),
    "sphere1280_mrhs": dict(n_tris=1280, axes=(1.0, 1.0, 1.0), k0=3.0,
                            eps_r=6.0 + 0j, mu_r=1.0 + 0j, mbj_block=100,
                            tol=1e-8, nrhs=128),
    "ellipsoid1280": dict(n_tris=1280, axes=(1.0, 0.8, 0.6), k0=3.0,
                          eps_r=3.0 + 0.1j, mu_r=1.0 + 0j, mbj_block=100,
                          tol=1e-12, nrhs=1),
}


def get_config(name: str) -> dict:
    c = dict(CONFIGS[name])
    c["name"] = name
    return c


def planewaves(name: str):
    """(khat[nrhs,3] float64, pol[nrhs,3] complex128) for a workload.

    Single-RHS workloads use khat = +z, pol = +x.  The multi-RHS workload
    draws 64 directions g ~ N(0, I3) from numpy's default_rng(0),
    normalises them, and pairs each with two polarisations:
    p1 = normalize(v_ref x khat), v_ref = x if |khat.z| > 0.9 else z,
    and p2 = khat x p1.
    """
    nrhs = CONFIGS[name]["nrhs"]
    if nrhs == 1:
        return (np.array([[0.0, 0.0, 1.0]]),
                np.array([[1.0 + 0j, 0.0, 0.0]], dtype=np.complex128))
    return planewave_set(nrhs // 2, seed=0)


def planewave_set(ndir: int, seed: int = 0):
    """2 ndir plane waves: ndir directions normalize(g), g ~ N(0, I3) from
    default_rng(seed), each with the two polarisations described above."""
    g = np.random.default_rng(seed).normal(size=(ndir, 3))
    kh = g / np.linalg.norm(g, axis=1, keepdims=True)
    khat = np.zeros((2 * ndir, 3))
    pol = np.zeros((2 * ndir, 3), dtype=np.complex128)
    for d in range(ndir):
        k = kh[d]
        vref = np.array([1.0, 0, 0]) if abs(k[2]) > 0.9 else np.array([0, 0, 1.0])
        p1 = np.cross(vref, k)
        p1 /= np.linalg.norm(p1)
        p2 = np.cross(k, p1)
        khat[2 * d] = k
        khat[2 * d + 1] = k
        pol[2 * d] = p1
        pol[2 * d + 1] = p2
    return khat, pol


def random_directions(n: int, seed: int) -> np.ndarray:
    """n unit vectors, normalised N(0, I3) draws from default_rng(seed)."""
    g = np.random.default_rng(seed).normal(size=(n, 3))
    return g / np.linalg.norm(g, axis=1, keepdims=True)


def cut_plane_directions(n: int = 360) -> np.ndarray:
    """r_j = (sin t_j, 0, cos t_j), t_j = j degrees: the xz-plane cut."""
    t = np.deg2rad(np.arange(n, dtype=np.float64))
    return np.stack([np.sin(t), np.zeros_like(t), np.cos(t)], axis=1)


def gradient_setup(n_nodes: int):
    """Seeded inputs of the gradient workload.

    Returns (d[n_nodes] float64 ~ N(0,1) from default_rng(1),
             nodes[16] int64 from default_rng(2).choice(n_nodes, 16)).
    """
    d = np.random.default_rng(1).normal(size=n_nodes)
    nodes = np.random.default_rng(2).choice(n_nodes, 16, replace=False)
    return d, np.sort(nodes).astype(np.int64)


# ---------------------------------------------------------------- spectra --
# Sweeps over the vacuum wavelength on one mesh (lengths in nm, free space,
# silver from workloads.materials).
#   spheroid_lspr  silver prolate spheroid, semi-axes 15, 15, 45 nm, cubed
#                  sphere n = 16 (3072 triangles, 6146 nodes, 24584
#                  unknowns); wave along +x, field along the major axis +z;
#                  the 131-wavelength grid of lspr_wavelengths(); block-Jacobi
#                  clusters of 100, GMRES to 1e-5.
#   sphere_lspr    silver sphere of radius 20 nm on the same cubed-sphere
#                  mesh and grid, the case with a closed form (Mie).
SPECTRA = {
    "spheroid_lspr": dict(cube_n=16, axes=(15.0, 15.0, 45.0), mbj_block=100, tol=1e-5),
    "sphere_lspr": dict(cube_n=16, axes=(20.0, 20.0, 20.0), mbj_block=100, tol=1e-5),
}


def spectrum_workload(name: str, lambdas=None):
    """(xyz, tri6, lam[npts] nm, k0[npts] 1/nm, eps_r[npts], khat[3], pol[3],
    settings) of a spectrum workload; lambdas overrides the grid."""
    from .materials import lspr_wavelengths, silver_eps
    from .meshes import cubesphere_p2
    c = dict(SPECTRA[name])
    xyz, tri = cubesphere_p2(c["cube_n"], c["axes"])
    lam = lspr_wavelengths() if lambdas is None else np.atleast_1d(np.asarray(lambdas, dtype=np.float64))
    khat = np.array([1.0, 0.0, 0.0])
    pol = np.array([0.0, 0.0, 1.0], dtype=np.complex128)
    return xyz, tri, lam, 2 * np.pi / lam, silver_eps(lam), khat, pol, c
