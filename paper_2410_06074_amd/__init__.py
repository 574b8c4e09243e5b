"""MI355X-native batched linear-ODE least-squares solve of Scalable Mechanistic
Neural Networks (the S-MNN solver): HIP kernels for gfx950 behind the C-ABI of
include/smnn.h, with a thin Python binding.

    from paper_2410_06074_amd import solve, Plan
"""
from ._lib import SmnnError, lib  # noqa: F401
from .solver import Plan, SmnnSolve, get_plan, solve  # noqa: F401
from .graph import CapturedSolve  # noqa: F401
from .tune import autotune  # noqa: F401

__all__ = ["Plan", "SmnnSolve", "SmnnError", "CapturedSolve", "autotune", "get_plan", "solve", "lib"]
