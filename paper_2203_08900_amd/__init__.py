"""MI355X-native structure-preserving spectral division for definite
pseudosymmetric matrices H = [[A, B], [-B, -A]] (Benner, Nakatsukasa, Penke,
arXiv 2203.08900).

The compute path is the HIP library ``libpseudosym.so`` (sources under
``csrc/``, C-ABI declared in ``include/pseudosym.h``); ``api`` is a thin ctypes
binding with the same entry-point names.  Importing the package does not load
the library; the first call into ``api`` does, and raises if it is missing.
"""
