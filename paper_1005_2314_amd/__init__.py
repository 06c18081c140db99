"""MI355X (gfx950) Wallace maximum-entropy normal generator.

The generator of R. P. Brent, "Some Comments on C. S. Wallace's Random Number
Generators" (Section 5): pools of normal variates renewed by 4x4 orthogonal
transforms with a chi-square rescale, computed by the HIP kernels of
``libwn.so`` behind the C ABI declared in ``include/wn.h``.

``wn`` is the thin ctypes binding; ``inputs`` holds the seeded synthetic
workloads.  Importing the package loads nothing; the library is loaded on
first use and its absence is an error (there is no fallback).
"""

__all__ = ["wn", "inputs"]
