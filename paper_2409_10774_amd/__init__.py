"""MI355X-native micropolar elastoplastic FFT-based solver (HIP, gfx950).

Submodules
  mp         ctypes binding of the C ABI (include/mp.h); loads _lib/libmp.so
  workloads  seeded synthetic inputs (phase maps, constants, load paths)
  build      in-tree hipcc build of the library

Nothing is imported eagerly, so the input generators can be used without a
built library; `paper_2409_10774_amd.mp` raises ImportError when it is missing.
"""
__all__ = ["mp", "workloads", "build"]
