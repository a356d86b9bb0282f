"""MI355X (gfx950) wall-distance solver: pseudo-time marching of the
Eikonal, Hamilton-Jacobi (standard, LAD, curvature-corrected) and Poisson
wall-distance equations with explicit/compact central differences and an
implicit filter, behind the C ABI of ``include/wd.h``.

Submodules: ``grids`` (seeded synthetic geometry), ``_lib`` (ctypes binding
of libwd.so with the C names), ``api`` (device placement helpers).  The
binding is loaded lazily so that ``grids`` can be used without a GPU.
"""
__all__ = ["grids", "api"]
__version__ = "1.0"
