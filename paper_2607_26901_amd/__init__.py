"""MI355X-native implementation of the CCFR hot path (candidates -> per-vertex
convex regions -> projection of XPBD-proposed displacements).

Modules:
  ccfr    ctypes binding of libccfr.so (the C ABI in include/ccfr.h)
  scenes  seeded synthetic workloads
  build   hipcc build of libccfr.so for gfx950
Importing the package touches neither the GPU nor the library.
"""
