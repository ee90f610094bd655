"""Divergence-distance fields and steepest-descent paths on MI355X (gfx950).

Hand-written HIP kernels behind the C ABI of ``include/dd.h`` (libdd.so);
this package is the thin Python binding over it.
"""

from ._lib import (DD_FORM_BF16X3, DD_FORM_F16X3, DD_FORM_F32, DD_FORM_NONE, DD_KL, DD_TV, DDError, LIB_PATH)
from .api import Context, Kernel, PATH_STATUS

__all__ = ["Context", "Kernel", "DDError", "DD_TV", "DD_KL", "DD_FORM_NONE", "DD_FORM_F32",
           "DD_FORM_F16X3", "DD_FORM_BF16X3", "PATH_STATUS", "LIB_PATH"]
