"""MI355X-native Barnes-Hut / direct-sum self-gravity (gfx950 HIP kernels).

Implements the gravity hot path of Ferrari, Lavagna & Blazquez, "A
parallel-GPU code for asteroid aggregation problems with angular particles"
(MNRAS 2020): octree Barnes-Hut accelerations rebuilt every step, the direct
N^2 sum, and a kick-drift-kick leapfrog. The kernels live in libbhx.so
(C ABI in include/bhx.h); this package only marshals torch tensors.
"""
from __future__ import annotations

__all__ = ["Context", "BHError", "load_library", "compute_accel", "compute_accel_direct",
           "step_leapfrog", "autotune", "gravity_dt_bound", "probe_fma", "rollout", "save_state",
           "load_state"]


def load_library():
    """Loads libbhx.so (raises if it has not been built)."""
    from . import _lib

    return _lib.load()


def __getattr__(name):
    if name in ("Context", "BHError", "compute_accel", "compute_accel_direct", "step_leapfrog",
                "autotune", "gravity_dt_bound", "probe_fma", "save_state", "load_state"):
        from . import api

        return getattr(api, name)
    if name == "rollout":
        from . import autograd

        return autograd.rollout
    raise AttributeError(name)
