"""MI355X-native Riemann-WCSPH hot path (SPHinXsys fluid scheme, arXiv 2010.12375).

`sphx` is the ctypes binding of the HIP library's C ABI (include/sphx.h);
`workloads` builds the seeded synthetic dam-break inputs.
"""
from . import workloads  # noqa: F401

__all__ = ["workloads", "sphx"]
