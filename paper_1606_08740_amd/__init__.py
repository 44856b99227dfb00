"""MI355X-native Alternating Anderson-Richardson (AAR) solver for stencil systems.

The solver itself lives in a HIP shared library behind a C ABI
(``include/aar.h``); :mod:`paper_1606_08740_amd.aar` is a thin ctypes binding
to it.  :mod:`paper_1606_08740_amd.inputs` holds the seeded synthetic
workloads.  Importing this package loads nothing: the binding loads the
library on first use and raises if it is missing.
"""
__version__ = "0.1.0"
