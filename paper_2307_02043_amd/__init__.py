"""MI355X-native hot path of the mini-batch quasi-Newton proximal method
(arXiv:2307.02043): the Lippmann-Schwinger mini-batch data-term gradient and
the weighted TV proximal mapping, as HIP kernels behind a C ABI
(include/bq.h) with this thin Python binding.

Importing the package loads libbq.so and raises ImportError when it has not
been built; nothing here falls back to CPU code.
"""
from ._lib import load as _load

_load()

from .api import BQError, LSContext, ProxInfo, QNInfo, QNIteration, SolveInfo, WProx  # noqa: E402
from .autograd import LSData, ls_data  # noqa: E402

__all__ = ["BQError", "LSContext", "LSData", "ProxInfo", "QNInfo", "QNIteration", "SolveInfo", "WProx",
           "ls_data"]
