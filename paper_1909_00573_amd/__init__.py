"""Next Event Backtracking hot path on MI355X (gfx950).

The compute runs in the HIP library ``libneb.so`` built from ``csrc/``;
``neb`` is its ctypes binding.
"""
from . import neb  # noqa: F401
from .neb import Renderer, DeviceOctree, NebError  # noqa: F401
