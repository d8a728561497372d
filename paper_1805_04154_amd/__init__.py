"""MI355X-native powersort (Munro & Wild, ESA 2018) for gfx950.

The sorting path lives in a HIP shared library with a C ABI
(``include/powersort_hip.h``); ``paper_1805_04154_amd.binding`` marshals torch
tensors into it.  Importing this package loads nothing; the binding loads the
library on first use and raises if it is missing.
"""
