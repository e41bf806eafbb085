"""Matrix-free non-nested multigrid for continuous Q_k elements on gfx950.

The compute path is the HIP library ``libnnmg.so`` (C ABI in include/nnmg.h);
this package only marshals arguments to it.  Importing the package fails if
the library has not been built.
"""

import torch  # noqa: F401  (its HIP runtime is the one the library binds to)

from ._lib import NNMGError, lib  # noqa: F401,E402

lib()  # load now: no silent fallback when the HIP library is missing

from .api import Context, Hierarchy, Level, Server, Ticket, Transfer, build_levels  # noqa: E402,F401
