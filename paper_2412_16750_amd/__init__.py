"""MI355X (gfx950) implementation of the differentiable IDM traffic simulator
of arXiv 2412.16750: forward simulation, reverse-mode gradient, trajectory
fitting and a learned warm start, all in hand-written HIP kernels behind the
C ABI of include/idm.h.

The HIP library must have been built (``__graft_entry__.build()``); importing
the compute entry points raises ImportError when it is missing.  There is no
CPU fallback.
"""
from ._lib import BOUND_CLAMP, BOUND_SOFTPLUS, EXPORTS, IdmError, load  # noqa: F401

__all__ = ["BOUND_CLAMP", "BOUND_SOFTPLUS", "EXPORTS", "IdmError", "load"]
