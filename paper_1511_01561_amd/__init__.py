"""MI355X-native hot path of the NUMA spectral-element dynamical core.

The compute path is the C-ABI library ``libnuma.so`` (hand-written HIP kernels
for gfx950, declared in ``include/numa.h``); ``paper_1511_01561_amd.numa`` is a
thin ctypes binding with the same names.  Importing this package does not load
the library; the binding loads it on first use and fails loudly if it is
missing.
"""
__all__ = ["inputs"]
