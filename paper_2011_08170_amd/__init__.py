"""libf2m: the F2M gradient descent procedure (arXiv 2011.08170) on MI355X.

The compute path is the HIP library libf2m.so behind the C ABI in
include/f2m.h; `paper_2011_08170_amd.f2m` is a thin ctypes binding over it.
Importing this package does not load the library; the binding loads it on
first use and raises if it is missing (there is no CPU fallback).
"""
__all__ = ["f2m", "instances"]
