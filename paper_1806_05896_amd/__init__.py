"""MI355X-native interior point solver for sparse, box-constrained
PDE-constrained optimal control (Pearson, Porcelli, Stoll, arXiv 1806.05896).

The solver lives in the HIP library libipmpde (C ABI, include/ipmpde.h);
this package is its thin Python binding.  PyTorch is used only for device
memory of the low-level operator calls and for streams."""
from .api import (Batch, Engine, Options, Problem, Stats, build_library, footprint_bytes,  # noqa: F401
                  library_path, use_torch_allocator)
from . import _lib  # noqa: F401
