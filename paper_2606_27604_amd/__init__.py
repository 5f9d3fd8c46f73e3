"""MI355X (gfx950) random-walk subsurface transport through a mixture of media.

Submodules:
  rw         - ctypes binding of the C ABI (include/rw.h), same entry-point names
  api        - tensor-level helpers (forward + finalize, adjoint, RWReflectance)
  workloads  - seeded synthetic inputs
  build      - in-tree hipcc build of librw.so

Importing the package loads nothing; the HIP library is loaded on first use and
its absence is an error (there is no CPU fallback).
"""
__all__ = ["rw", "api", "workloads", "build"]
