"""MI355X-native 1D PIC-MCC positive-column engine.

The particle path (gather, push, collisions, radial sink, compaction, sort,
deposit, field solve) runs in hand-written gfx950 HIP kernels behind the C
ABI in include/pc.h; this package holds the in-tree build of that library
and a thin ctypes binding.
"""
from . import native  # noqa: F401

__all__ = ["native", "Column"]


def __getattr__(name):
    if name == "Column":
        from .column import Column
        return Column
    raise AttributeError(name)
