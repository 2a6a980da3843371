"""MI355X-native H-matrix LU (hot path of arXiv 1911.07531).

Submodules:
  inputs  seeded synthetic workloads (no method arithmetic)
  hm      ctypes binding of libhm.so (build_htree, h_assemble, h_lu, h_solve, h_matvec)
  build   in-tree build of libhm.so for gfx950
"""
