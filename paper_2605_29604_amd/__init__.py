"""MI355X (gfx950) round-synchronous priority MIS: the hot path of TC-MIS.

Subpackages / modules:
  tcmis     -- ctypes binding of libtcmis.so (C ABI in include/tcmis.h)
  gen       -- seeded synthetic graph inputs (shared with the CPU oracle)
  build_lib -- compiles csrc/*.hip for gfx950 into libtcmis.so
"""
