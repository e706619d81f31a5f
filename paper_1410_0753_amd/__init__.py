"""MI355X-native split-step shallow-water solver (Cliffs method, arXiv 1410.0753).

Submodules
  clf    -- ctypes binding of the HIP library libclf.so (include/clf.h)
  synth  -- seeded synthetic inputs (bathymetry, deformations, gauges)
  build  -- hipcc build of libclf.so for gfx950
"""
