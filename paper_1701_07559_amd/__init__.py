"""MI355X (gfx950) solver for the Moebius domain-wall operator of arXiv:1701.07559.

Submodules:
  mdwf    -- ctypes binding of the C ABI in include/mdwf.h (loads libmdwf.so)
  inputs  -- seeded synthetic gauge fields and sources
  build   -- hipcc build of libmdwf.so

The binding is not imported here so that the input generators stay usable on
machines without the built library.
"""
