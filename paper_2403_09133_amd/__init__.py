"""MI355X (gfx950) implementation of the LoRADS hot path.

The compute lives in the HIP library `liblorads.so` (sources in `csrc/`, C ABI in
`include/lorads.h`); `lorads` is its ctypes binding.
"""
from . import lorads  # noqa: F401
from .lorads import Context, Gnn, default_options, gram, load  # noqa: F401
