"""MI355X (gfx950) coherent beamformer.

``bf``     -- Python binding of the C ABI in ``include/bf.h`` (libbf.so).
``synth``  -- seeded synthetic inputs (shared with the tests and the bench).
``build``  -- in-tree hipcc build of libbf.so.
"""
from . import bf, synth  # noqa: F401

__all__ = ["bf", "synth"]
