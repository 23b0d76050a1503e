"""MI355X (gfx950) absolute-offset LZ77: host encoder + HIP match-phase decoder.

The native library ``liblz.so`` (sources in ``csrc/``, ABI in ``include/lz.h``)
does all the work; ``lz`` is its ctypes binding.
"""
from . import lz  # noqa: F401
