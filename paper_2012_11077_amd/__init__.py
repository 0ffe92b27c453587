"""Integral-image 2D CA-CFAR on AMD Instinct MI355X (gfx950).

The hot path (integral image, eq. 3; eight-corner box sums, eq. 4; threshold
T = alpha * A, eq. 2; decision CUT > T, eq. 1 of arXiv 2012.11077) runs in
hand-written HIP kernels behind the C ABI declared in ``include/cfar2d.h``
(``libcfar2d.so``).  ``paper_2012_11077_amd.cfar2d`` is the thin ctypes
binding; ``paper_2012_11077_amd.synth`` draws seeded synthetic maps.

Importing the package loads nothing; the binding loads the library on first
use and raises if it is missing.
"""
__all__ = ["cfar2d", "synth"]
