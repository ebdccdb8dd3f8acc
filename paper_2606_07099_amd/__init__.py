"""Batched Newton-Raphson AC power flow and its implicit adjoint on AMD
Instinct MI355X (gfx950), behind the C ABI of ``include/sable_pf.h``.

The HIP library ``libsablepf.so`` is built in-tree by
``python -m paper_2606_07099_amd.build``; importing the Python API requires
it (there is no CPU fallback).
"""
from ._lib import LIB_PATH, PFError, lib  # noqa: F401
from .pf import PFTemplate, symbolic_analyze, ybus_from_branches  # noqa: F401

__all__ = ["PFTemplate", "PFLayer", "PFLayerFunction", "symbolic_analyze", "ybus_from_branches",
           "PFError", "lib", "LIB_PATH"]


def __getattr__(name):
    if name in ("PFLayer", "PFLayerFunction"):
        from . import layer
        return getattr(layer, name)
    raise AttributeError(name)
