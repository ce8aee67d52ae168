"""F-COO sparse tensor operations for AMD Instinct MI355X (gfx950).

The unified method of "A Unified Optimization Approach for Sparse Tensor
Operations on GPUs": the F-COO format (Sec. IV-B) with one-shot,
segmented-scan SpMTTKRP and SpTTM kernels (Sec. IV-C, IV-D) driving CP-ALS
(Algorithm 1), plus gradient-based sparse CP.  The computation lives in
libfcoo.so (hand-written HIP for gfx950 behind the C ABI of include/fcoo.h);
this package marshals arguments and uses torch for device memory and streams.
"""
from . import _lib  # noqa: F401  (fails loudly if libfcoo.so is missing)
from ._lib import FcooError  # noqa: F401
from .tensor import Tensor  # noqa: F401
from .cp import CPAtNonzeros, CPMSELoss, cp_als  # noqa: F401

__all__ = ["Tensor", "FcooError", "cp_als", "CPAtNonzeros", "CPMSELoss"]
