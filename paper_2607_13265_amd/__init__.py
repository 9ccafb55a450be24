"""MI355X (gfx950) differentiable polarized path tracing.

Monte Carlo path tracing in Mueller-Stokes calculus with reverse-mode gradients by path
replay backpropagation and cached suffix radiance (no Mueller matrix inversion), behind the
C ABI of include/ppt.h.  Every step of the hot path runs in the hand-written HIP kernels of
libppt.so; this package only marshals arguments.
"""
from ._lib import LIB_PATH, PPTError, lib  # noqa: F401
from .core import FLAG_NO_NEE, VIEW_DTYPE, Plan, Scene, debug_rng  # noqa: F401
from .autograd import PolarizedRender, render  # noqa: F401
