"""MI355X (gfx950) library for symmetry-adapted spin-1/2 exact
diagonalisation: sector bases, matrix-free y = H x and Lanczos, in HIP.

The Python layer is a ctypes binding of ``include/xdg.h`` (see ``xdg``);
the library is built in-tree by ``paper_2505_02901_amd.build``.
"""
from .xdg import *  # noqa: F401,F403
from .xdg import Basis, Hamiltonian, XdgError, lib  # noqa: F401
