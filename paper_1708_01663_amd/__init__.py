"""MI355X (gfx950) implementation of the CISOR reconstruction hot path.

The HIP library ``libcisor.so`` (built in-tree by ``build.py``) implements the
relaxed-FISTA iteration of arXiv 1708.01663: batched FFT-BiCGSTAB
Lippmann-Schwinger solves, receiver projection on the matrix cores, the
Prop. 1 adjoint gradient and the FGP total-variation prox.  ``cisor.Cisor``
and ``cisor.Fista`` are the Python front end; importing this package does not
load the library until a context is created.
"""

__all__ = ["Cisor", "Fista", "SolveOpts"]


def __getattr__(name):
    if name in __all__:
        from . import cisor
        return getattr(cisor, name)
    raise AttributeError(name)
