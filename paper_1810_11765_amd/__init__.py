"""MI355X-native SMMO object heap (DynaSOAr method, arXiv 1810.11765).

The compute path is the HIP library ``libsmmo.so`` built from ``csrc/``; the
Python modules only marshal arguments for its C-ABI (``include/smmo.h``).
"""
