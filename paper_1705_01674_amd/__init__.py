"""MI355X-native SG-WLS filtering (Semi-Global Weighted Least Squares,
Liu et al., ICCV 2017, arXiv 1705.01674).

The filter runs in hand-written HIP kernels for gfx950 behind the C ABI of
``include/sgwls.h``; this package is the thin Python binding.  Importing
``paper_1705_01674_amd.ops`` loads the in-tree ``libsgwls.so`` and raises if it
has not been built.
"""
__all__ = ["ops", "synth"]
