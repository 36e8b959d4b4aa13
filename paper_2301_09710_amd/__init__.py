"""MI355X-native (gfx950) rotation-based SPECT projector pair.

  spect   -- ctypes binding of libspect.so (the HIP kernels behind include/spect.h)
  synth   -- seeded synthetic inputs (phantoms, attenuation maps, PSFs)
  build   -- compiles libspect.so in-tree with hipcc

Importing the package does not load the shared library; ``spect.load()`` or
the first call does, and raises if it has not been built.
"""
__all__ = ["spect", "synth", "build"]
