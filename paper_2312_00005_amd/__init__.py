"""MI355X-native Burton-Miller BEM / multilevel FMM (arXiv 2312.00005 hot path).

``bemfmm`` is the ctypes binding of the HIP library ``libbemfmm.so``; build it
with ``python -m paper_2312_00005_amd.build``.  Importing ``bemfmm`` fails if
the library is missing -- there is no CPU fallback.
"""

__all__ = ["bemfmm"]
