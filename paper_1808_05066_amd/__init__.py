"""Entropy-variable hybridized DG hot path on MI355X (gfx950).

The compute lives in the HIP library ``lib/libhdg.so`` (C ABI in
``include/hdg.h``); ``hdg.Plan`` is a thin binding that passes torch device
pointers and the current stream.  Importing this package does not import torch
or load the library; both happen on first use, and a missing library raises.
"""
from ._lib import LIB_PATH, HdgError, load  # noqa: F401


def __getattr__(name):
    if name in ("Plan", "selftest"):
        from . import hdg
        return getattr(hdg, name)
    raise AttributeError(name)
