"""MI355X (gfx950) solver for the per-increment pseudo-transient
elasto-plastic solve: HIP kernels behind the C ABI of include/ep.h, loaded
through the ctypes binding in `ep`."""
from . import ep  # noqa: F401

__all__ = ["ep"]
