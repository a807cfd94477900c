"""Exact integer time-difference estimation on AMD Instinct MI355X (gfx950).

The estimator of Ueno, Sato and Ono (quantize both signals with monotone
integer maps, correlate exactly in integer arithmetic, take the argmax;
Algorithm 1 of the paper) as hand-written HIP kernels behind the C ABI of
``libtde.so`` (``include/tde.h``). ``paper_2509_19974_amd.tde`` is the ctypes
binding; ``paper_2509_19974_amd.build`` compiles the library.
"""
__all__ = ["tde", "build"]
