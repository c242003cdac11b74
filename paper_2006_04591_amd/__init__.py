"""MI355X-native (gfx950) digital shearlet filter bank.

The transform of "tfShearlab" (Andrade-Loarca, Kutyniok): Algorithm 1
(decomposition), Algorithm 2 (reconstruction) and the adjoint, as hand-written
HIP kernels behind the C ABI in include/shear.h. This package is the thin
Python binding over that library.
"""
from ._binding import (
    EXPORTED,
    LIB_PATH,
    ShearError,
    ShearletSystem,
    ShrinkNet,
    delta_schedule,
    design_spectra,
    load_library,
)

from .autograd import ShearletLayer, ShearletTransform
from .batched import UnevenInpainter

__all__ = ["EXPORTED", "LIB_PATH", "ShearError", "ShearletLayer", "ShearletSystem", "ShearletTransform", "delta_schedule",
           "ShrinkNet", "UnevenInpainter", "design_spectra", "load_library"]
