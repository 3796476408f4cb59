"""c3tod: the TOD step of a Commander3-style Gibbs sampler on AMD MI355X (gfx950).

Huffman pointing decode, sky projection, correlated-noise constrained
realisation and map binning as hand-written HIP kernels behind a C-ABI
(``include/c3tod.h``, ``libc3tod.so``); this package is its Python binding.
"""
from ._lib import LIB_PATH, LibraryMissing  # noqa: F401


def load():
    """Load the native library (raises LibraryMissing if it is not built)."""
    from . import _lib
    return _lib.load()
