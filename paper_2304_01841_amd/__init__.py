"""MI355X-native LArTPC signal-simulation hot path (arXiv:2304.01841, Sec. 2).

The compute path is the HIP library ``libwcsim.so`` (C ABI in
``include/wcsim.h``); :mod:`paper_2304_01841_amd.wcsim` is its thin binding.
Importing this package loads nothing; importing the binding loads the library
and raises if it is missing.
"""
__all__ = ["wcsim", "workloads"]
