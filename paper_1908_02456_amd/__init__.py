"""MI355X (gfx950) time stepper for the 3D Schroedinger equation with discrete
DtN absorbing boundary conditions (Wu & Li, arXiv:1908.02456).

The compute path is the HIP library ``libabc_dtn.so`` (C ABI in
include/abc_dtn.h); :mod:`.solver` binds it to torch tensors.  Importing this
package loads nothing; :class:`Solver` loads the library on first use and
raises if it has not been built.
"""

__all__ = ["Solver"]


def __getattr__(name):
    if name == "Solver":
        from .solver import Solver
        return Solver
    raise AttributeError(name)
