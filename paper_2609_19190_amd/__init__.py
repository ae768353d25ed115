"""MI355X-native radiomic spatial mapping (gfx950 HIP kernels behind a C ABI).

Modules:
  binding  thin ctypes binding of libflashrad.so (include/fr.h)
  synth    seeded synthetic CT/PET inputs (no method arithmetic)
  build    compiles libflashrad.so in-tree for gfx950
Nothing is imported eagerly, so importing the package needs no GPU.
"""
__all__ = ["binding", "synth", "build"]
