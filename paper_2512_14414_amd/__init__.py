"""Single-layer (nested) CTMRG for iPEPS on MI355X (arXiv:2512.14414).

The computation lives in libctm.so (HIP kernels for gfx950, C ABI in
include/ctm.h); ``CTM`` is its thin Python binding.
"""
from .binding import CTM, CTMError, EXPORTED, LIB, LIB_PATH, PRECISIONS, torch_allocator  # noqa: F401
from .autograd import CTMEnergy  # noqa: F401
from .binding import Surrogate, energy_objective, lbfgs, lbfgs_params, python_objective  # noqa: F401
