"""MI355X-native fourth-order cut-cell multigrid solver (HIP for gfx950).

``ccgmg`` binds the C interface of ``libccgmg.so`` (declared in
include/ccgmg.h); ``autograd`` wraps the solve as a torch.autograd.Function.
"""
from .ccgmg import CcgmgError, Solver, default_options, lib  # noqa: F401
