"""ctypes declarations of libashrt's C ABI (include/ashrt.h).

Argument marshalling only.  Loading fails loudly when the library has not
been built: there is no fallback implementation.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libashrt.so")

ASHRT_OK = 0
ASHRT_E_INVALID_ARG = -1
ASHRT_E_UNSUPPORTED_SIZE = -2
ASHRT_E_HIP = -3
ASHRT_E_NONFINITE = -4
ASHRT_E_OOM = -5
ASHRT_E_NOT_IMPLEMENTED = -6
ASHRT_E_WORKSPACE = -7

OP_FORWARD, OP_ADJOINT, OP_INVERT, OP_FISTA = 0, 1, 2, 3

# kernel families for ashrt_profile_enable / ashrt_profile_read
K_XFFT_MODEL, K_XFFT_DATA, K_ROWS_FWD, K_ROWS_FIN, K_XINV_DATA, K_ROWS_ADJ, K_XINV_MODEL, \
    K_VECTOR, K_REDUCE, K_SELECT = range(10)
K_COUNT = 10


class AshrtDesc(C.Structure):
    _fields_ = [
        ("nt", C.c_int32), ("nx", C.c_int32), ("ntp", C.c_int32), ("nxp", C.c_int32),
        ("dt", C.c_double), ("dx", C.c_double),
        ("npanel", C.c_int32),
        ("vel", C.POINTER(C.c_double)),
        ("tau0_samples", C.POINTER(C.c_int32)),
        ("panel_scale", C.POINTER(C.c_double)),
        ("fmin_hz", C.c_double), ("fmax_hz", C.c_double),
        ("half_width", C.c_int32),
        ("wavelet_amp", C.POINTER(C.c_double)),
        ("x_pos", C.POINTER(C.c_double)),
    ]


class IrlsParams(C.Structure):
    _fields_ = [
        ("p", C.c_int32), ("q", C.c_int32), ("n_outer", C.c_int32), ("n_inner", C.c_int32),
        ("b_r", C.c_double), ("b_m", C.c_double), ("tol", C.c_double), ("eps_floor_rel", C.c_double),
        ("freeze_eps", C.c_int32),
        ("cg_graph", C.c_int32),
    ]


class UnetDesc(C.Structure):
    _fields_ = [("cin", C.c_int32), ("pout", C.c_int32), ("base", C.c_int32)]


class UnetTrainParams(C.Structure):
    _fields_ = [("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double),
                ("weight_decay", C.c_double), ("lam_w", C.c_double)]


class Tuning(C.Structure):
    _fields_ = [("tile_model", C.c_int32), ("tile_data", C.c_int32), ("nchunk", C.c_int32)]


class FistaParams(C.Structure):
    _fields_ = [("n_iter", C.c_int32), ("n_power", C.c_int32), ("mu", C.c_double), ("mu_rel", C.c_double),
                ("lip_safety", C.c_double)]


class FistaReport(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("lipschitz", C.c_double), ("mu", C.c_double),
                ("misfit", C.c_double), ("l1", C.c_double), ("objective", C.c_double)]


class IrlsReport(C.Structure):
    _fields_ = [
        ("status", C.c_int32), ("outer_done", C.c_int32),
        ("inner", C.c_int32 * 64),
        ("misfit", C.c_double * 64), ("huber", C.c_double * 64),
        ("eps_r", C.c_double * 64), ("eps_m", C.c_double * 64),
    ]


class PlanInfo(C.Structure):
    _fields_ = [
        ("nt", C.c_int32), ("nx", C.c_int32), ("ntp", C.c_int32), ("nxp", C.c_int32),
        ("npanel", C.c_int32), ("half_width", C.c_int32),
        ("jlo", C.c_int32), ("jhi", C.c_int32), ("kmax", C.c_int32), ("nchunk", C.c_int32),
        ("tile_model", C.c_int32), ("tile_data", C.c_int32),
        ("ws_forward", C.c_size_t), ("ws_adjoint", C.c_size_t),
        ("ws_invert_q2", C.c_size_t), ("ws_invert_q1", C.c_size_t),
    ]


_lib = None


ABI_VERSION = 5  # struct layouts below match include/ashrt.h at this version


def lib():
    """Load libashrt.so (once).  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"libashrt.so not found at {LIB_PATH}; build it with "
            "`python -c 'import __graft_entry__ as g; g.build()'` (hipcc, gfx950)")
    L = C.CDLL(LIB_PATH)
    vp, i32, sz = C.c_void_p, C.c_int32, C.c_size_t
    P_desc, P_prm, P_rep = C.POINTER(AshrtDesc), C.POINTER(IrlsParams), C.POINTER(IrlsReport)
    sig = {
        "ashrt_desc_default": (None, [P_desc]),
        "irls_params_default": (None, [P_prm]),
        "ashrt_desc_validate": (C.c_int, [P_desc]),
        "irls_params_validate": (C.c_int, [P_prm]),
        "ashrt_plan_create": (C.c_int, [P_desc, C.c_int, C.POINTER(vp)]),
        "ashrt_plan_create_tuned": (C.c_int, [P_desc, C.POINTER(Tuning), C.c_int, C.POINTER(vp)]),
        "ashrt_batch_plan_create_tuned": (C.c_int, [P_desc, i32, C.POINTER(Tuning), C.c_int, C.POINTER(vp)]),
        "ashrt_autotune": (C.c_int, [P_desc, C.c_int, i32, C.POINTER(Tuning), C.POINTER(C.c_double)]),
        "fista_params_default": (None, [C.POINTER(FistaParams)]),
        "fista_invert": (C.c_int, [vp, C.POINTER(FistaParams), vp, vp, vp, vp, C.POINTER(FistaReport), vp, sz, vp]),
        "ashrt_blend": (C.c_int, [vp, i32, i32, i32, vp, vp, i32, vp]),
        "ashrt_deblend": (C.c_int, [vp, i32, i32, i32, vp, i32, vp, i32, vp]),
        "ashrt_resort": (C.c_int, [vp, i32, i32, i32, vp, vp]),
        "ashrt_td_forward": (C.c_int, [vp, vp, vp, vp, vp]),
        "ashrt_td_adjoint": (C.c_int, [vp, vp, vp, vp, vp]),
        "ashrt_plan_destroy": (None, [vp]),
        "ashrt_plan_get_info": (C.c_int, [vp, C.POINTER(PlanInfo)]),
        "ashrt_workspace_bytes": (C.c_int, [vp, C.c_int, P_prm, C.POINTER(sz)]),
        "ashrt_forward": (C.c_int, [vp, vp, vp, vp, vp, sz, vp]),
        "ashrt_forward_noalloc": (C.c_int, [vp, vp, vp, vp, vp]),
        "ashrt_vec_stats": (C.c_int, [vp, vp, C.c_int64, C.c_double, C.c_int32, vp, vp]),
        "ashrt_weight_target": (C.c_int, [vp, vp, C.c_int64, C.c_double, vp, vp]),
        "ashrt_vec_scale": (C.c_int, [vp, C.c_int64, C.c_double, vp, vp]),
        "ashrt_adjoint": (C.c_int, [vp, vp, vp, vp, vp, sz, vp]),
        "robust_invert": (C.c_int, [vp, P_prm, vp, vp, vp, vp, vp, P_rep, vp, sz, vp]),
        "ashrt_batch_plan_create": (C.c_int, [P_desc, i32, C.c_int, C.POINTER(vp)]),
        "ashrt_batch_plan_destroy": (None, [vp]),
        "ashrt_batch_layout": (C.c_int, [vp] + [C.POINTER(C.c_int64)] * 6),
        "ashrt_batch_workspace_bytes": (C.c_int, [vp, C.c_int, P_prm, C.POINTER(sz)]),
        "ashrt_forward_batched": (C.c_int, [vp, vp, vp, vp, vp, sz, vp]),
        "ashrt_adjoint_batched": (C.c_int, [vp, vp, vp, vp, vp, sz, vp]),
        "robust_invert_batched": (C.c_int, [vp, P_prm, vp, vp, vp, vp, vp, P_rep, vp, sz, vp]),
        "ashrt_status_string": (C.c_char_p, [C.c_int]),
        "ashrt_last_error": (C.c_char_p, []),
        "ashrt_abi_version": (C.c_int, []),
        "ashrt_profile_enable": (C.c_int, [C.c_uint32]),
        "ashrt_profile_read": (C.c_int, [C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int]),
        "ashrt_kernel_name": (C.c_char_p, [C.c_int]),
        # learned warm start (include/unet.h)
        "unet_create": (C.c_int, [C.POINTER(UnetDesc), C.c_int, C.POINTER(vp)]),
        "unet_destroy": (None, [vp]),
        "unet_param_count": (C.c_int64, [vp]),
        "unet_set_params": (C.c_int, [vp, vp, C.c_int64]),
        "unet_get_params": (C.c_int, [vp, vp, C.c_int64]),
        "unet_workspace_bytes": (C.c_int, [vp, i32, i32, i32, i32, C.POINTER(sz)]),
        "unet_forward": (C.c_int, [vp, vp, i32, i32, i32, vp, vp, vp, sz, vp]),
        "unet_loss_grad": (C.c_int, [vp, vp, vp, vp, i32, i32, i32, C.c_double, vp, vp, vp, sz, vp]),
        "unet_train_step": (C.c_int, [vp, C.POINTER(UnetTrainParams), vp, vp, vp, i32, i32, i32, vp, vp, sz,
                                      vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    if L.ashrt_abi_version() != ABI_VERSION:
        raise ImportError(f"libashrt.so has ABI {L.ashrt_abi_version()}, the binding expects {ABI_VERSION}; rebuild it")
    _lib = L
    return L


class AshrtError(RuntimeError):
    def __init__(self, status, where):
        L = lib()
        msg = L.ashrt_last_error().decode(errors="replace")
        super().__init__(f"{where}: {L.ashrt_status_string(status).decode()} ({status}): {msg}")
        self.status = status


def check(status, where):
    if status != ASHRT_OK:
        raise AshrtError(status, where)
    return status
