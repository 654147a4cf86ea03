"""mbem: MI355X (gfx950) library for the nodal P2 Mueller boundary-element
method (arXiv 2604.21181): Galerkin fill, Morton block-Jacobi GMRES solve,
far field.  The compute path is the HIP library ``libmbem.so`` built by
``paper_2604_21181_amd.build``; ``paper_2604_21181_amd.mbem`` is its ctypes
binding.  Importing the package itself loads nothing.
"""
__all__ = ["build", "mbem"]
