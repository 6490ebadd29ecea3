"""MI355X-native 4-D spectral-convolution FNO block (arXiv 2211.12709, Sec. IV-C).

The compute lives in the HIP library libfno_mi355x.so (C-ABI, include/fno_mi355x.h);
`paper_2211_12709_amd.fno` is its Python binding.  Importing this package does
not load the library; `from paper_2211_12709_amd import fno` does, and raises
if it is missing.
"""
__all__ = ["fno", "inputs"]
