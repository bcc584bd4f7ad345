"""MI355X (gfx950) implementation of the radiative-transfer step of Jiang,
Stone & Davis (2014): HIP kernels behind the C ABI of ``include/rt.h``.

``rt`` is the ctypes binding (same names as the C entry points), ``Solver``
a marshalling helper that keeps one problem's arrays in device memory,
``build`` compiles ``librt.so``.
"""
from . import rt  # noqa: F401


def __getattr__(name):
    if name == "Solver":
        from .solver import Solver
        return Solver
    if name == "build":
        from .build import build
        return build
    raise AttributeError(name)
