"""MI355X (gfx950) resource-stressor suite and victim-colocation harness.

The device library is libcoloc.so (C ABI in include/coloc.h); `coloc` is its
Python binding.  Nothing here computes on the host: a missing library is an
error, never a fallback.
"""
from . import coloc  # noqa: F401

__all__ = ["coloc"]
