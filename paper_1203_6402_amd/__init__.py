"""k-means|| (Bahmani et al., "Scalable K-Means++") on AMD MI355X (gfx950).

The compute path is ``libkmpar.so`` (hand-written HIP kernels behind a C ABI
declared in ``include/kmpar.h``); ``paper_1203_6402_amd.kmpar`` is the thin
Python binding.  Importing this package loads nothing; importing the binding
loads the library and fails loudly if it has not been built.
"""
__version__ = "0.1.0"
