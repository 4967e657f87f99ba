"""MI355X-native infinite-cell Clenshaw-Curtis Spectral Quadrature (SQ) hot path.

The compute path lives in a C-ABI shared library built from ``csrc/`` (HIP for
gfx950); ``sq`` is the thin ctypes binding over it and ``workloads`` generates
the seeded synthetic cells.  Importing the package does not load the library:
``paper_2006_03697_amd.sq.load()`` does, and raises if it is missing.
"""

__all__ = ["workloads", "sq"]
