"""MI355X-native critical-curve and caustic finder (after Weisenbach 2025,
arXiv 2506.02121): C-ABI library libmlcc.so (HIP, gfx950) and its binding.

Submodules:
  fields  seeded synthetic star fields and the named workloads (no GPU needed)
  mlcc    ctypes binding of libmlcc.so; raises on import if it is not built
  build   compiles libmlcc.so for gfx950
"""
