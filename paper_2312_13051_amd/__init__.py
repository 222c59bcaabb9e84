"""berryhip: batched Wilson-loop engine for MI355X (gfx950).

The hot path lives in the HIP library ``libberryhip.so`` (see
``include/berryhip.h``); ``_lib`` is its ctypes binding and ``pipeline``
chains the C-ABI calls for whole k-planes.
"""
from . import _lib  # noqa: F401
from ._lib import Context, BerryError  # noqa: F401
