"""MI355X-native Schwarzschild black-hole ray tracer (arXiv 2507.16165).

The compute path is the C-ABI library ``libbh.so`` (hand-written HIP for
gfx950); ``api`` holds the thin ctypes binding.  Importing the package does
not load the library; the first call does, and fails loudly if it is missing.
"""
__all__ = ["inputs"]
