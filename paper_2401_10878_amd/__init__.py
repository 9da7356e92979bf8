"""MI355X-native HLBM + discrete-contact time step (arXiv 2401.10878).

Submodules:
  workloads  seeded synthetic inputs (parameters, particle scenes)
  hlbm       ctypes binding of the HIP library libhlbm.so (C-ABI in include/hlbm.h)

Nothing is imported eagerly, so the input module can be used without a GPU.
"""
__all__ = ["workloads", "hlbm"]
