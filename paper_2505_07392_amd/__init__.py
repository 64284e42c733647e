"""IGR compressible-Euler hot path for AMD MI355X (gfx950).

The solver lives in the HIP library ``libigr.so`` (C ABI declared in
``include/igr.h``); :mod:`paper_2505_07392_amd.igr` is its thin ctypes
binding and :mod:`paper_2505_07392_amd.inputs` defines seeded synthetic
workloads.  Importing the package loads nothing; the binding loads the
library on first use and raises if it is missing.
"""
