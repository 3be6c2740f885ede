"""MI355X (gfx950) library for the interpolation-based imaging operators of
three-dimensional optoacoustic tomography: the projector H = D G, its exact
adjoint H^T and filtered backprojection, as HIP kernels behind the C ABI of
include/oat.h.  `Plan` (in .oat) binds them to torch tensors."""
from .synth import Geometry  # noqa: F401

__all__ = ["Geometry", "Plan", "OatError"]


def __getattr__(name):
    if name in ("Plan", "OatError"):
        from . import oat
        return getattr(oat, name)
    raise AttributeError(name)
