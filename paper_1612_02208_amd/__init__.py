"""MI355X multigrid solver for the Stokes-immersed-boundary saddle-point system
(Bhalla, Knepley, Adams, Guy, Griffith: geometric multigrid with additive
Schwarz and Schur-complement smoothers for semi-implicit IB).

The computation lives in libibmg.so (HIP for gfx950, C ABI in
include/ibmg.h); this package only marshals arguments.  Importing the
package does not load the library; constructing ``StokesIB`` does, and fails
loudly when it is missing.
"""

__all__ = ["StokesIB", "StokesIBBatch", "IbmgError"]


def __getattr__(name):
    if name in ("StokesIB", "StokesIBBatch", "IbmgError"):
        from . import solver
        return getattr(solver, name)
    raise AttributeError(name)
