"""MI355X-native TTNS one-site TDVP library (HIP kernels behind a C-ABI).

The compute path lives in libttns.so (include/ttns.h); ``ttns`` is the thin
ctypes binding.  Importing this package does not load the library.
"""
