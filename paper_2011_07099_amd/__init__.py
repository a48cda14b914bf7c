"""Natively periodic FMM on MI355X (gfx950).

The solver lives in the HIP/C++ shared library ``libpfmm.so`` (C ABI declared in
``include/pfmm.h``); ``paper_2011_07099_amd.pfmm`` is its thin ctypes binding.
Importing this package loads nothing; the library is opened on first use.
"""
