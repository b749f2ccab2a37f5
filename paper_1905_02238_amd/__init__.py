"""libfsmi: MI355X-native FSMI (Shannon mutual information for range beams).

The compute lives in the HIP library ``libfsmi.so`` behind the C-ABI declared
in ``include/libfsmi.h``; ``paper_1905_02238_amd.fsmi`` is the thin ctypes
binding.  Importing this package does not load the library; the first call
into ``fsmi`` does, and raises if it has not been built.
"""
__all__ = ["fsmi", "workloads"]
