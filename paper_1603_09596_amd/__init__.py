"""kd-GeRaF query path on MI355X (gfx950).

The forest build and every step of the query path run in the native library
``libgeraf.so`` (C-ABI declared in include/geraf.h); ``geraf`` is its thin
ctypes binding.  Importing this package loads nothing: ``geraf`` loads the
library on first use and raises if it has not been built.
"""
__all__ = ["geraf", "workloads"]
