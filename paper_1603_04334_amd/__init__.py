"""MI355X Chebyshev-filter hot path of real-space Kohn-Sham DFT (arXiv:1603.04334).

Submodules: ``inputs`` (seeded synthetic clusters), ``binding`` (ctypes
binding of libsparcfilter.so), ``build`` (hipcc build of the library).
Nothing is loaded at import time.
"""
