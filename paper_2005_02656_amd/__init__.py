"""MI355X-native SPH time step (arXiv 2005.02656).

* ``paper_2005_02656_amd.sph``    -- ctypes binding of the HIP library libsph.so
  (include/sph.h); it raises on first use if the library is not built: there is
  no CPU fallback.
* ``paper_2005_02656_amd.inputs`` -- seeded synthetic workloads (no method
  arithmetic).
* ``paper_2005_02656_amd.build``  -- compiles libsph.so for gfx950.
"""
