"""Adaptive-Multilevel BDDC on one MI355X (HIP library + thin Python binding).

The numeric path lives in libambddc.so (C ABI in include/ambddc.h); this
package only marshals arguments.  Importing it does not load the library;
``Handle`` does, and fails loudly when it has not been built.
"""
from .solver import Handle, SolveResult, analyze  # noqa: F401
from ._lib import AmbddcError, LIB_PATH, EXPORTED  # noqa: F401

__all__ = ["Handle", "SolveResult", "analyze", "AmbddcError", "LIB_PATH", "EXPORTED"]
