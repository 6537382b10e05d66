"""MI355X (gfx950) overlap-and-save fast convolution.

Paper: Adamek, Dimoudi, Giles, Armour, "GPU Fast Convolution via the
Overlap-and-Save Method in Shared Memory".  The C ABI is include/ols.h; the
kernels are in csrc/; this package marshals arguments from PyTorch tensors.
"""

from ._lib import OLSError, lib  # noqa: F401

__all__ = ["OLSError", "lib", "OLSPlan", "OLSConv", "OLSConvFunction", "OLSBatch", "ols_conv"]


def __getattr__(name):
    if name in ("OLSPlan", "OLSConv", "OLSConvFunction", "OLSBatch", "ols_conv", "calibration_copy"):
        from . import ols as _ols
        return getattr(_ols, name)
    raise AttributeError(name)
