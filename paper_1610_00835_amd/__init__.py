"""MI355X-native volume-integral solver for isotropic radiative transport.

The compute path lives in the HIP library ``libertvie.so`` behind the C ABI
declared in ``include/ertvie.h``; ``ertvie`` is its thin ctypes binding.
Importing the package loads nothing: the library is opened on first use.
"""
__all__ = ["inputs", "ertvie"]
