"""MI355X-native explicit finite-difference wave-propagation hot path.

The compute lives in ``libfd.so`` (hand-written HIP for gfx950 behind the
C ABI declared in ``include/fd.h``); ``paper_2312_13094_amd.fd`` is the thin
ctypes binding to it.  Importing this package does not load the library, so
``synth`` (the seeded input generators) is usable on hosts without a GPU.
"""
