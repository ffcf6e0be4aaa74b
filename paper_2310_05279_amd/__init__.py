"""MI355X (gfx950) implementation of the D3(BJ) dispersion correction.

The computation lives in the HIP library ``libd3.so`` (sources in
``csrc/``, C ABI in ``include/d3.h``); ``d3`` is its ctypes binding.
"""

from . import d3  # noqa: F401
from .d3 import D3, D3Error  # noqa: F401
