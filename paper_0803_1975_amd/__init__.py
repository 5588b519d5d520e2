"""Q-adic compressed modular matrix multiplication on AMD MI355X (gfx950).

The compute lives in the HIP library libqmm.so (C ABI in include/qmm.h); the
module `qmm` is its Python binding.  Build the library with
`paper_0803_1975_amd.build.build()`.
"""
from . import qmm  # noqa: F401

__all__ = ["qmm"]
