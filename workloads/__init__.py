"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package only *produces inputs*: surface meshes, material/incidence
settings and seeded random vectors.  It holds none of the discretisation's
arithmetic (no quadrature, no kernels, no frames), so the oracle and the HIP
path can both consume it without sharing any computation.
"""
from .meshes import cubesphere_p2, icosphere_p2, mesh_counts, uv_sphere_p2
from .configs import CONFIGS, SPECTRA, get_config, planewaves, random_directions, spectrum_workload
from .materials import lspr_wavelengths, silver_eps

__all__ = ["cubesphere_p2", "icosphere_p2", "mesh_counts", "uv_sphere_p2", "CONFIGS", "SPECTRA",
           "get_config", "planewaves", "random_directions", "spectrum_workload",
           "lspr_wavelengths", "silver_eps"]
