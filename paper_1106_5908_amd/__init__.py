"""MI355X-native CRS sparse matrix-vector multiplication (libspmv).

The compute path lives in ``csrc/`` (gfx950 HIP kernels and a C++ runtime
behind the C interface of ``include/spmv.h``); ``spmv`` is its ctypes
binding.  Importing this package loads nothing; the library is loaded on the
first call of a binding function and an ImportError is raised if it has not
been built.
"""
