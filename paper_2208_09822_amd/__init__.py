"""Input-aware adaptive tiling (IAAT) small GEMM on MI355X (gfx950).

The compute path is the HIP library ``libiaat.so`` behind the C ABI declared
in ``include/iaat.h``; ``paper_2208_09822_amd.iaat`` is its thin ctypes
binding.  Importing this package loads nothing; the binding loads the library
on first use and raises if it has not been built.
"""
__all__ = ["iaat", "inputs"]
