"""MI355X (gfx950) implementation of the PALM-KQR hot path.

* ``kqr``    -- ctypes binding of libkqr (include/kqr.h); loads the library on
               first use and raises if it was not built.
* ``inputs`` -- seeded synthetic workloads.
* ``build``  -- compiles the HIP sources in csrc/ into libkqr.so.

Importing the package loads nothing; the library is opened by the first call.
"""
__all__ = ["kqr", "inputs", "build"]
