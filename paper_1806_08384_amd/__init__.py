"""Exact selectivity by a COUNT scan on MI355X (gfx950).

The library itself is ``libsel.so`` (C ABI in include/sel.h); ``sel`` is its
Python binding.  Importing ``sel`` fails if the library is not built.
"""
__all__ = ["sel"]
