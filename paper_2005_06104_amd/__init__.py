"""GSE-TDVP1 hot path for MI355X (gfx950).

The compute lives in the HIP shared library built from ``csrc/`` and exposed
through the C-ABI declared in ``include/tdvp.h``; ``tdvp`` is a thin ctypes
binding with the same entry-point names.  Importing this package does not load
the library; ``paper_2005_06104_amd.tdvp`` does.
"""
