"""MI355X-native QR-based CP-ALS (CP-ALS-QR) hot path.

The compute lives in ``libcpqr.so`` (hand-written HIP for gfx950 behind a
C ABI declared in ``include/cpqr.h``).  ``paper_2112_10855_amd.cpqr`` is the
thin ctypes binding with the same entry-point names; it loads the library on
first use and raises if it is missing.  ``synth`` holds the seeded input
generators.
"""
