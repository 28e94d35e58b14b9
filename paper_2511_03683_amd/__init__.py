"""MI355X-native e-ph collision integral (arXiv 2511.03683, Eq. 2).

The compute path is libephbte.so (HIP, gfx950) behind the C ABI in
include/ephbte.h; this package is its ctypes binding plus autograd wrappers.
Importing it loads the library and fails if it has not been built.
"""
from .binding import (F32, F64, EphbteError, Plan, autotune, build_channels, collision_integral,
                      collision_integral_noalloc,
                      collision_vjp, collision_vjp_nph, destroy, iterate_transport, kernel_timing, last_error,
                      layout_host, load_library, phonon_rate, phonon_rate_vjp, plan_bytes, plan_info,
                      rt_adjoint, rt_adjoint_coupled, rt_step, rt_step_coupled, set_field, set_tuning, status_string, update_g2)

load_library()

__all__ = ["F32", "F64", "EphbteError", "Plan", "autotune", "build_channels",
           "collision_integral", "collision_integral_noalloc", "collision_vjp", "collision_vjp_nph", "destroy", "iterate_transport", "kernel_timing",
           "last_error",
           "layout_host", "load_library", "phonon_rate", "phonon_rate_vjp", "plan_bytes", "plan_info",
           "rt_adjoint", "rt_adjoint_coupled",
           "rt_step", "rt_step_coupled", "set_field", "set_tuning", "status_string", "update_g2"]
