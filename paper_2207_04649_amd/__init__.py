"""MI355X-native exact density-peaks clustering (Amagata and Hara, arXiv 2207.04649).

The compute path is a C-ABI shared library of hand-written HIP kernels for
gfx950 (``csrc/``); :mod:`.dpc` is its thin Python binding.  Importing the
package does not load the library: the first call does, and raises if it is not
built.
"""
from . import inputs  # noqa: F401

__all__ = ["inputs"]
