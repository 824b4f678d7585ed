"""MI355X (gfx950) state-vector gate engine (mpiQulacs method, one GPU).

``binding`` is the ctypes layer over libqs (include/qs.h); ``state.State`` is a torch-backed handle wrapper.
"""
from . import binding
from .binding import (QS_C128, QS_C64, QSError, qs_alloc, qs_apply_controlled, qs_apply_diag, qs_apply_gate,
                      qs_copy_in, qs_copy_out, qs_free, qs_fused_swap, qs_get_info, qs_init_zero, qs_last_error,
                      qs_norm, qs_probs, qs_renormalize, qs_scale, qs_sync)
from .state import State

__all__ = ["binding", "State", "QSError", "QS_C128", "QS_C64", "qs_alloc", "qs_free", "qs_apply_gate",
           "qs_apply_diag", "qs_apply_controlled", "qs_fused_swap", "qs_probs", "qs_init_zero", "qs_copy_in",
           "qs_copy_out", "qs_sync", "qs_scale", "qs_norm", "qs_renormalize", "qs_get_info", "qs_last_error"]
