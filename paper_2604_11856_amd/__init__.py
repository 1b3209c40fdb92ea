"""MI355X-native line-by-line + ray-march radiation hot path (arXiv 2604.11856).

Submodules:
  synth  -- seeded synthetic workloads (inputs only)
  lrt    -- ctypes binding of the C-ABI library liblrt.so (HIP kernels, gfx950)
"""
