"""ctypes declarations of the C ABI in ``include/hofks.h``.

Loading fails loudly when ``libhofks.so`` has not been built: there is no
fallback implementation.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhofks.so")

OK, EINVAL, ESIZE, EDEVICE, ENONPHYS, ESTATE = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "HOFKS_OK", -1: "HOFKS_EINVAL", -2: "HOFKS_ESIZE", -3: "HOFKS_EDEVICE",
                -4: "HOFKS_ENONPHYS", -5: "HOFKS_ESTATE"}

# every symbol include/hofks.h declares
SYMBOLS = [
    "hofks_workspace_size", "hofks_create", "hofks_set_tau", "hofks_set_state_macro",
    "hofks_set_state_f", "hofks_step", "hofks_sync", "hofks_read_moments", "hofks_read_f",
    "hofks_read_counters", "hofks_kernel_timing", "hofks_dt", "hofks_batch_workspace_size",
    "hofks_batch_create", "hofks_batch_tube_flags", "hofks_autotune", "hofks_last_error", "hofks_destroy",
    "hofks_closure_enable", "hofks_closure_disable", "hofks_closure_snapshot", "hofks_closure_stats",
    "hofks_mlp_nparam", "hofks_mlp_packed_bytes", "hofks_mlp_pack", "hofks_mlp_forward",
    "hofks_mlp_grad", "hofks_mlp_adam", "hofks_state_bytes", "hofks_read_state", "hofks_write_state",
    "hofks_read_tail_substeps", "hofks_set_euler_launches", "hofks_mlp_grad_work_bytes",
    "hofks_closure_prepare_work_bytes", "hofks_closure_prepare", "hofks_mlp_fold_scales",
    "hofks_closure_train_step", "hofks_closure_set_weights", "hofks_mlp_grad_noalloc",
    "hofks_stream_probe", "hofks_set_launch_config", "hofks_batch_set_launch_config",
]


class GridDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n_cells", ctypes.c_int * 3), ("dx", ctypes.c_double),
                ("n_vel", ctypes.c_int), ("dv", ctypes.c_double), ("bc", ctypes.c_int * 3),
                ("precision", ctypes.c_int), ("scheme", ctypes.c_int), ("dt", ctypes.c_double),
                ("splitting", ctypes.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_1212_0204_amd.build` "
            "(hipcc --offload-arch=gfx950); there is no CPU fallback")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp, i, d, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    dp = P(ctypes.c_double)
    L.hofks_workspace_size.argtypes = [P(GridDesc), P(sz)]
    L.hofks_create.argtypes = [P(GridDesc), vp, sz, vp, P(vp)]
    L.hofks_set_tau.argtypes = [vp, d]
    L.hofks_set_state_macro.argtypes = [vp, dp, dp, dp]
    L.hofks_set_state_f.argtypes = [vp, dp, sz]
    L.hofks_step.argtypes = [vp, i]
    L.hofks_sync.argtypes = [vp]
    L.hofks_read_moments.argtypes = [vp, dp]
    L.hofks_read_f.argtypes = [vp, dp, sz]
    L.hofks_read_counters.argtypes = [vp, P(i), P(ctypes.c_long)]
    L.hofks_kernel_timing.argtypes = [vp, i, dp, P(i)]
    L.hofks_read_tail_substeps.argtypes = [vp, P(ctypes.c_long)]
    L.hofks_set_euler_launches.argtypes = [vp, i]
    L.hofks_batch_workspace_size.argtypes = [P(GridDesc), i, P(sz)]
    L.hofks_batch_create.argtypes = [P(GridDesc), dp, i, vp, sz, vp, P(vp)]
    L.hofks_batch_tube_flags.argtypes = [vp, P(i)]
    L.hofks_autotune.argtypes = [vp, i, ctypes.c_char_p, P(i)]
    L.hofks_dt.argtypes = [vp]
    L.hofks_dt.restype = d
    L.hofks_last_error.argtypes = [vp]
    L.hofks_last_error.restype = ctypes.c_char_p
    L.hofks_destroy.argtypes = [vp]
    L.hofks_destroy.restype = None
    L.hofks_state_bytes.argtypes = [vp, P(sz)]
    L.hofks_read_state.argtypes = [vp, vp, sz]
    L.hofks_write_state.argtypes = [vp, vp, sz]
    L.hofks_closure_enable.argtypes = [vp, vp, d, d]
    L.hofks_closure_disable.argtypes = [vp]
    L.hofks_closure_snapshot.argtypes = [vp, vp, vp]
    L.hofks_closure_stats.argtypes = [vp, P(ctypes.c_long), P(ctypes.c_ulonglong)]
    L.hofks_mlp_nparam.restype = i
    L.hofks_mlp_packed_bytes.restype = sz
    L.hofks_mlp_pack.argtypes = [vp, vp, vp]
    L.hofks_mlp_forward.argtypes = [vp, vp, vp, ctypes.c_long, vp]
    L.hofks_mlp_grad.argtypes = [vp, vp, vp, vp, ctypes.c_long, vp, vp, vp, sz, vp]
    L.hofks_mlp_grad_noalloc.argtypes = [vp, vp, vp, vp, ctypes.c_long, vp, vp, vp]
    L.hofks_mlp_grad_work_bytes.argtypes = [ctypes.c_long]
    L.hofks_mlp_grad_work_bytes.restype = sz
    L.hofks_closure_prepare_work_bytes.argtypes = [ctypes.c_long]
    L.hofks_closure_prepare_work_bytes.restype = sz
    L.hofks_closure_prepare.argtypes = [vp, vp, ctypes.c_long, ctypes.c_float, vp, vp, vp, vp, vp,
                                        sz, vp]
    L.hofks_mlp_fold_scales.argtypes = [vp, vp, vp]
    f = ctypes.c_float
    L.hofks_closure_train_step.argtypes = [vp, vp, vp, vp, vp, vp, vp, ctypes.c_long, f, f, f, f,
                                           i, vp, vp, vp, sz, vp]
    L.hofks_closure_set_weights.argtypes = [vp, vp, sz]
    L.hofks_stream_probe.argtypes = [i, vp, vp, sz, vp]
    L.hofks_set_launch_config.argtypes = [vp, i, i, i]
    L.hofks_batch_set_launch_config.argtypes = [vp, i, i]
    L.hofks_mlp_adam.argtypes = [vp, vp, vp, vp, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                 ctypes.c_float, i, vp]
    _lib = L
    return L
