"""MI355X-native fused element-wise expression trees and reductions
(the data-parallel hot path of the Bandicoot GPU library, arXiv:2308.03120).

The compute path is libcoot_mi355x.so (HIP, gfx950); this package is its
ctypes binding.  Importing the package does not load the library; the first
call does, and fails loudly if it has not been built.
"""
from . import coot  # noqa: F401
from .coot import CootError  # noqa: F401

__all__ = ["coot", "CootError"]
