"""MI355X-native orthogonalization-free Rayleigh-Ritz (OFRR) library.

The method (Xu, Zhang, Chen, Saad and Xi, arXiv 2505.00281) runs in the HIP
library libofrr.so behind the C ABI of include/ofrr.h; `ofrr` is its thin
Python binding.
"""
from . import ofrr  # noqa: F401
from .ofrr import Context, make_plan, dense_matrix, csr_matrix, OfrrError  # noqa: F401
