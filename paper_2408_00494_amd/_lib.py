"""ctypes binding of libbssmppi (the C ABI declared in include/bssmppi.h).

Argument marshalling only: every step of the solve runs in the library's HIP kernels.  The
library is loaded from this package directory; when it has not been built the import of the
binding fails loudly instead of falling back to anything else.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbssmppi.so")

BSS_OK, BSS_E_INVAL, BSS_E_NOMEM, BSS_E_DEVICE, BSS_E_STATE, BSS_E_NUMERIC = range(6)
BSS_OUT_CONTROLS = 1
BSS_OUT_BELIEFS = 2
STATUS_NAMES = {0: "BSS_OK", 1: "BSS_E_INVAL", 2: "BSS_E_NOMEM", 3: "BSS_E_DEVICE",
                4: "BSS_E_STATE", 5: "BSS_E_NUMERIC"}


class BssError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class BssParams(C.Structure):
    """Mirror of ``bss_params`` (field order and types must match the header)."""
    _fields_ = [
        ("m", C.c_double), ("Iz", C.c_double), ("lf", C.c_double), ("lr", C.c_double),
        ("Cf", C.c_double), ("Cr", C.c_double), ("mu", C.c_double), ("g", C.c_double),
        ("v_min", C.c_double), ("dt", C.c_double),
        ("steer_max", C.c_double), ("accel_max", C.c_double),
        ("sigma_eps", C.c_double * 2), ("sigma_w", C.c_double * 3),
        ("K", C.c_int32), ("M", C.c_int32), ("T", C.c_int32),
        ("delta", C.c_double), ("gamma", C.c_double),
        ("backoff", C.c_int32),
        ("lambda_", C.c_double), ("gamma_u", C.c_double), ("v_goal", C.c_double),
        ("q_vx", C.c_double), ("q_vy", C.c_double), ("q_r", C.c_double), ("q_ey", C.c_double),
        ("q_epsi", C.c_double), ("C_cbf", C.c_double), ("C_obs", C.c_double),
        ("phi_scale", C.c_double),
        ("ell_a", C.c_double), ("ell_b", C.c_double), ("half_width", C.c_double),
        ("shield_iters", C.c_int32), ("shield_gmin", C.c_double), ("shield_fd", C.c_double),
        ("seed", C.c_uint64),
        ("lanes", C.c_int32),
        ("belief", C.c_int32),
        ("crn", C.c_int32),
        ("sigma_w_speed", C.c_double),
        ("n_obs", C.c_int32),
        ("obs", C.c_double * 12),
        ("local_repair", C.c_int32),
        ("n_con", C.c_int32),
        ("con_a", C.c_double * 24),
        ("con_b", C.c_double * 4),
        ("vehicle", C.c_int32),
        ("Rw", C.c_double), ("Iw", C.c_double), ("T_max", C.c_double),
        ("pac_B", C.c_double), ("pac_C", C.c_double), ("pac_D", C.c_double),
        ("pac_E", C.c_double),
        ("track_len", C.c_double), ("kappa_amp", C.c_double),
        ("n_sub", C.c_int32),
    ]


class BssAllocator(C.Structure):
    _fields_ = [("alloc", C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)),
                ("release", C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)),
                ("user", C.c_void_p)]


class BssBuffers(C.Structure):
    _fields_ = [("v", C.c_void_p), ("u", C.c_void_p), ("mom", C.c_void_p), ("S", C.c_void_p),
                ("stats", C.c_void_p), ("x0", C.c_void_p), ("Sigma0", C.c_void_p),
                ("v_shift", C.c_int32), ("con_var", C.c_void_p)]


class BssInfo(C.Structure):
    _fields_ = [("S_min", C.c_double), ("Z", C.c_double), ("ess", C.c_double),
                ("n_finite", C.c_int32), ("lanes", C.c_int32), ("ppl", C.c_int32),
                ("split", C.c_int32), ("dcbf_violations", C.c_int32), ("kernel_ms", C.c_float),
                ("records_on_chip", C.c_int32)]


# every exported symbol of include/bssmppi.h
EXPORTS = [
    "bss_params_default", "bss_validate", "bss_backoff", "bss_create", "bss_set_stream",
    "bss_solve", "bss_solve_async", "bss_step_shift", "bss_set_outputs", "bss_get_buffers",
    "bss_get_controls",
    "bss_set_controls", "bss_set_solve_index", "bss_get_solve_index", "bss_get_info",
    "bss_timing_enable", "bss_timing_read", "bss_set_lanes", "bss_destroy", "bss_last_error",
    "bss_dev_philox", "bss_dev_normals", "bss_dev_disturbance", "bss_dev_model_step", "bss_dev_model_step8", "bss_dev_sdf", "bss_dev_score",
    "bss_dev_update_workspace", "bss_dev_update", "bss_dev_repair", "bss_set_shape",
    "bss_batch_create", "bss_batch_states", "bss_batch_set_states", "bss_batch_copy_states", "bss_batch_solve",
    "bss_batch_capture", "bss_batch_tune", "bss_batch_set_grid", "bss_batch_info",
    "bss_batch_set_member_ppl", "bss_batch_member_shape", "bss_batch_destroy",
    "bss_server_config_default", "bss_server_create", "bss_server_submit", "bss_server_pump",
    "bss_server_poll", "bss_server_drain", "bss_server_get_controls", "bss_server_set_controls",
    "bss_server_vehicle_state", "bss_server_replay", "bss_server_destroy",
    "bss_solve_noalloc", "bss_noalloc_scratch_bytes",
]


class BssServerConfig(C.Structure):
    """Mirror of ``bss_server_config``."""
    _fields_ = [("n_vehicles", C.c_int32), ("T", C.c_int32), ("K_max", C.c_int32),
                ("M_max", C.c_int32), ("ppl", C.c_int32), ("n_streams", C.c_int32),
                ("max_batch", C.c_int32), ("hbm_budget", C.c_uint64)]


class BssCompletion(C.Structure):
    """Mirror of ``bss_completion``."""
    _fields_ = [("req", C.c_int64), ("vehicle", C.c_int32), ("status", C.c_int32),
                ("u0", C.c_double * 2), ("t_done", C.c_double)]


def _declare(lib):
    P = C.POINTER(BssParams)
    vp = C.c_void_p
    i32, i64, u32, u64 = C.c_int32, C.c_int64, C.c_uint32, C.c_uint64
    d = C.c_double
    sig = {
        "bss_params_default": (None, [P]),
        "bss_validate": (i32, [P]),
        "bss_backoff": (i32, [P, C.POINTER(d)]),
        "bss_create": (i32, [P, C.POINTER(BssAllocator), vp, C.POINTER(vp)]),
        "bss_set_stream": (i32, [vp, vp]),
        "bss_solve": (i32, [vp, C.POINTER(d), vp, C.POINTER(d), C.POINTER(BssInfo)]),
        "bss_solve_async": (i32, [vp, vp, vp]),
        "bss_step_shift": (i32, [vp]),
        "bss_set_outputs": (i32, [vp, i32]),
        "bss_get_buffers": (i32, [vp, C.POINTER(BssBuffers)]),
        "bss_get_controls": (i32, [vp, vp]),
        "bss_set_controls": (i32, [vp, vp]),
        "bss_set_solve_index": (i32, [vp, u32]),
        "bss_get_solve_index": (i32, [vp, C.POINTER(u32)]),
        "bss_get_info": (i32, [vp, C.POINTER(BssInfo)]),
        "bss_timing_enable": (i32, [vp, i32]),
        "bss_timing_read": (i32, [vp, C.POINTER(d), C.POINTER(i32)]),
        "bss_set_lanes": (i32, [vp, i32]),
        "bss_destroy": (None, [vp]),
        "bss_last_error": (C.c_char_p, []),
        "bss_dev_philox": (i32, [u64, vp, vp, i64, vp]),
        "bss_dev_normals": (i32, [u64, vp, vp, i64, vp]),
        "bss_dev_disturbance": (i32, [u64, u32, i32, i32, i32, i32, i32, i32, vp, vp, vp]),
        "bss_solve_noalloc": (i32, [P, u32, vp, vp, vp, vp, vp, vp]),
        "bss_noalloc_scratch_bytes": (C.c_size_t, [P]),
        "bss_dev_model_step": (i32, [P, vp, vp, vp, i64, vp]),
        "bss_dev_model_step8": (i32, [P, vp, vp, vp, i64, vp]),
        "bss_dev_sdf": (i32, [d, d, vp, vp, i64, vp]),
        "bss_dev_score": (i32, [P, vp, vp, vp, vp, vp]),
        "bss_dev_update_workspace": (C.c_size_t, [i32, i32]),
        "bss_dev_update": (i32, [P, vp, vp, vp, vp, vp, vp]),
        "bss_dev_repair": (i32, [P, vp, vp, vp, i64, vp]),
        "bss_set_shape": (i32, [vp, i32, i32, i32]),
        "bss_batch_create": (i32, [C.POINTER(vp), i32, i32, i32, C.POINTER(vp)]),
        "bss_batch_states": (i32, [vp, C.POINTER(vp)]),
        "bss_batch_set_states": (i32, [vp, vp]),
        "bss_batch_copy_states": (i32, [vp, vp]),
        "bss_batch_solve": (i32, [vp]),
        "bss_batch_capture": (i32, [vp]),
        "bss_batch_tune": (i32, [vp, C.POINTER(i32)]),
        "bss_batch_set_grid": (i32, [vp, i32]),
        "bss_batch_set_member_ppl": (i32, [vp, C.POINTER(i32)]),
        "bss_batch_member_shape": (i32, [vp, i32, C.POINTER(i32), C.POINTER(i32)]),
        "bss_batch_info": (i32, [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]),
        "bss_batch_destroy": (None, [vp]),
        "bss_server_config_default": (None, [C.POINTER(BssServerConfig)]),
        "bss_server_create": (i32, [C.POINTER(BssServerConfig), P, C.POINTER(vp)]),
        "bss_server_submit": (i32, [vp, i32, i32, i32, d, vp, C.POINTER(i64)]),
        "bss_server_pump": (i32, [vp, C.POINTER(i32)]),
        "bss_server_poll": (i32, [vp, C.POINTER(BssCompletion), i32]),
        "bss_server_drain": (i32, [vp]),
        "bss_server_get_controls": (i32, [vp, i32, vp]),
        "bss_server_set_controls": (i32, [vp, i32, vp]),
        "bss_server_vehicle_state": (i32, [vp, i32, C.POINTER(u32), C.POINTER(i64)]),
        "bss_server_replay": (i32, [vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp]),
        "bss_server_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build the HIP library first (__graft_entry__.build() or "
                "python paper_2408_00494_amd/build.py)")
        _lib = _declare(C.CDLL(LIB_PATH))
    return _lib


def check(status):
    if status != BSS_OK:
        msg = lib().bss_last_error()
        raise BssError(status, msg.decode() if msg else "")
    return status


def params_from_problem(problem: dict) -> BssParams:
    """Fill a ``BssParams`` from a problem dict (keys as in ``workloads.default_problem``)."""
    p = BssParams()
    lib().bss_params_default(C.byref(p))
    for name, _ in BssParams._fields_:
        key = "lambda" if name == "lambda_" else name
        if key not in problem:
            continue
        val = problem[key]
        if name in ("sigma_eps", "sigma_w", "obs", "con_a", "con_b"):
            arr = getattr(p, name)
            for i, x in enumerate(val):
                arr[i] = float(x)
        else:
            setattr(p, name, type(getattr(p, name))(val))
    return p
