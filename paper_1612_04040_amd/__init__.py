"""Narrow-band first-order upwind level-set update on AMD MI355X (gfx950).

The compute path is the C-ABI library ``libls.so`` built from ``csrc/``; the
``ls`` module binds it with ctypes.  Importing this package loads nothing: the
library is opened on first use and a missing library is an error, never a
fallback.
"""
__all__ = ["ls", "workloads", "metrics"]
