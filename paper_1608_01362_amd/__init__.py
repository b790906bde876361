"""MI355X (gfx950) CSR segmenting for pull-direction graph traversal.

The compute path is libcagra.so (hand-written HIP, C ABI in include/cagra.h);
``cagra`` is its ctypes binding and iteration driver.
"""
from . import cagra  # noqa: F401

__all__ = ["cagra"]
