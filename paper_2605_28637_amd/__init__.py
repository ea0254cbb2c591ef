"""MI355X (gfx950) restricted open-shell Kohn-Sham plane-wave hot path.

Submodules:
  inputs  -- seeded synthetic problem descriptions (no method arithmetic)
  roks    -- ctypes binding of libroks.so (include/roks.h)
  build   -- builds libroks.so in-tree with hipcc

Importing the package loads nothing; ``roks.lib()`` loads the shared library
and raises if it has not been built.
"""
__all__ = ["inputs", "roks", "build"]
