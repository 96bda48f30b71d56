"""MI355X-native pseudo-spectral elastic seismogram simulation (arXiv 1705.04874).

Submodules:
  inputs   seeded synthetic workloads (models, receivers, sources, events)
  binding  ctypes binding of the HIP library libpstd3d.so (include/pstd3d.h)
  build    hipcc build of the library for gfx950

The binding is imported lazily so that the input generators can be used on a
machine without the built library.
"""
__all__ = ["inputs", "binding", "build"]
