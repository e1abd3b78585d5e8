"""Statically condensed GL-DGSEM implicit-step solve on AMD Instinct MI355X.

The solver lives in the HIP library libscdg.so (C ABI: include/scdg.h); this
package is its Python binding.  Importing the package does not load the
library; `Plan(...)` does, and raises ImportError when it has not been built.
"""
from ._lib import EXPORTED, LIB_PATH, ScdgError, load  # noqa: F401
from .plan import Plan  # noqa: F401
from .dg import DgResidual  # noqa: F401

__all__ = ["Plan", "DgResidual", "ScdgError", "load", "LIB_PATH", "EXPORTED"]
