"""MI355X (gfx950) E-A-HALS: extrapolated accelerated HALS for NMF
(Ang & Gillis, arXiv 1805.06604) as hand-written HIP behind a C ABI.

The Python layer only marshals arguments to libnmf.so; see binding.py.
"""
from .binding import (FLAG_BETA_STAR, FLAG_BETABAR_LAST_ACCEPTED, FLAG_CMP_LAST_ACCEPTED,  # noqa: F401
                      PHASES, Batch,
                      EXPORTS, LIB_PATH, Format, Inner, NMFError, Params, Prod, Result,
                      Solver, Status, XDtype, lib, make_params, solve, solve_noalloc)
