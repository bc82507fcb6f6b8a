"""Sliced tensor-network contraction with shared-work reuse on AMD MI355X.

The contraction itself runs in ``libtnmi.so`` (C ABI in include/tn.h, HIP
kernels for gfx950).  This package is its thin Python face:

* ``binding.Plan``       plan / contract / backward through the C ABI;
* ``autograd.Amplitude`` torch.autograd.Function over tn_contract(_backward).
"""

from .binding import Plan, TnError, permute  # noqa: F401
