"""Row-wise decomposed multi-dimensional FFTs (Duy & Ozaki) on AMD MI355X.

The product is the native library ``libfftrw.so`` (C ABI in include/fftrw.h):
host C++ for the decomposition maps, communication amounts and transpose
orders; HIP kernels for gfx950 for the FFT passes and transposes.  The Python
module ``fftrw`` is a ctypes binding with the same entry-point names.
Importing this package loads nothing; ``fftrw.lib()`` loads the library and
fails loudly if it has not been built.
"""
__all__ = ["fftrw", "inputs"]
