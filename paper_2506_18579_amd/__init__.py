"""MI355X-native batched HF ionospheric ray tracing (RTM-GD hot path).

Submodules:
  synth  -- seeded synthetic grids, fans and request streams (inputs only)
  rtgd   -- thin ctypes binding of the HIP C-ABI library ``librtgd.so``
  build  -- compiles the HIP library for gfx950
"""
__all__ = ["synth", "rtgd", "build"]
