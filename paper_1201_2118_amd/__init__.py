"""MI355X (gfx950) incompressible Navier-Stokes stencil step.

The step (predictor, Poisson right-hand side, red-black SOR, projection,
ghost fill) runs in hand-written HIP kernels behind the C ABI of
``include/ns.h`` (``libns.so``); ``abi`` binds it with the same names and
``solver`` adds torch-based conveniences.
"""
from . import abi  # noqa: F401

__all__ = ["abi", "Solver", "NSRollout", "make_params"]


def __getattr__(name):
    if name in ("Solver", "NSRollout", "make_params"):
        from . import solver
        return getattr(solver, name)
    raise AttributeError(name)
