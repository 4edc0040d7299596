"""MI355X-native Wilson-Dirac operator and CG solvers (libbsm).

Submodules:
  bsm     ctypes binding of the C ABI in include/bsm.h (loads libbsm.so)
  inputs  seeded synthetic gauge and spinor fields
  build   in-tree hipcc build of libbsm.so

Importing the package loads nothing; the HIP library is loaded on the first
call and raises if it has not been built.
"""
