"""MI355X (gfx950) particle-in-cell hot path: gather + relativistic Boris +
Esirkepov deposit on supercell-sorted FP32 frames, Yee field update, and a
Monte Carlo ionisation step.  The computation lives in the HIP library
libpic.so behind the C ABI of include/pic.h; this package only loads it."""
from ._capi import PicError, load  # noqa: F401
from .pic import Pic  # noqa: F401
