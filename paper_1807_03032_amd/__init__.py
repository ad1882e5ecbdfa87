"""MI355X (gfx950) finite-difference wave-equation operators: isotropic
acoustic and TTI pseudo-acoustic leapfrog time marching with a damping layer,
sparse source injection and receiver interpolation (arXiv 1807.03032).

Submodules:
  fdw        ctypes binding of the C ABI in include/fdw.h (libfdw.so)
  workloads  seeded synthetic inputs (models, coordinates, wavelets)
  build      hipcc build of libfdw.so

Importing the package loads nothing; `fdw.load()` loads the HIP library and
fails loudly if it has not been built.
"""
__all__ = ["fdw", "workloads", "build"]
