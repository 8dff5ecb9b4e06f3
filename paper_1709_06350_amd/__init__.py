"""MI355X-native nonlinear multigrid for initial-density reconstruction.

The computation lives in the HIP library libmr.so (C ABI in include/mr.h); ``mr`` is its thin
ctypes binding and ``autograd`` wraps the solve and its adjoint as a torch.autograd.Function.
"""
from . import mr  # noqa: F401
from . import autograd  # noqa: F401
from .mr import Context, Info, MRError, solve_batched  # noqa: F401
