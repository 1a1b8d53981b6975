"""MI355X-native semi-coherent Hough search for neutron stars in binary orbits.

The HIP library ``libbsh.so`` (C ABI in include/bsh.h) runs every step of the
search; ``paper_1904_04873_amd.bsh`` is the torch-facing binding with the same
names.  Importing this package does not load the library; the first call does,
and fails loudly if it has not been built.
"""
from . import _native  # noqa: F401

__version__ = "1.0.0"


def load():
    """Load libbsh.so (raises ImportError if it is not built)."""
    return _native.load()
