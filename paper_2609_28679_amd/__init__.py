"""MI355X-native lattice Boltzmann collide-and-stream library (HIP kernels behind a C ABI).

Submodules:
  binding  ctypes binding of liblbm.so (Lattice, Trainer)
  build    hipcc build of liblbm.so for gfx950
  inputs   seeded synthetic initial fields
"""
