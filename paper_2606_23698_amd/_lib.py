"""ctypes loader of libobfft.so.  Fails loudly when the HIP library is missing."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libobfft.so")

_lib = None


class ObfftError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status})" if what else status_string(status))


class PlanInfo(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("substrate", ctypes.c_int), ("r", ctypes.c_int),
                ("moduli", ctypes.c_int32 * 16), ("log2M", ctypes.c_double),
                ("budget_bits", ctypes.c_double), ("p", ctypes.c_int * 3), ("q", ctypes.c_int * 3),
                ("S", ctypes.c_int), ("S_frac", ctypes.c_int), ("n", ctypes.c_int64 * 3),
                ("workspace_bytes", ctypes.c_size_t)]


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("substrate", ctypes.c_int), ("p", ctypes.c_int * 3),
                ("q", ctypes.c_int * 3), ("n_moduli_override", ctypes.c_int),
                ("moduli_override", ctypes.POINTER(ctypes.c_int32)), ("reduction", ctypes.c_int),
                ("group_block", ctypes.c_int), ("axis_order", ctypes.c_int * 3), ("reserved", ctypes.c_int * 3)]


class TapsLayout(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int) for n in ("P", "Z", "E", "n_E", "zhat", "R", "n_R", "stride")]


class CrtConstants(ctypes.Structure):
    _fields_ = [("r", ctypes.c_int), ("S", ctypes.c_int), ("S_frac", ctypes.c_int),
                ("log2M", ctypes.c_double), ("moduli", ctypes.c_int32 * 16),
                ("M", ctypes.c_uint32 * 4), ("u", (ctypes.c_uint32 * 4) * 16),
                ("w", ctypes.c_uint64 * 16)]


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2606_23698_amd.build.build() "
                          "(there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    P = ctypes.POINTER
    sigs = {
        "obfft_options_default": (None, [P(Options)]),
        "obfft_plan_create": (i32, [P(vp), i64, i64, i64, P(Options)]),
        "obfft_plan_destroy": (i32, [vp]),
        "obfft_plan_info": (i32, [vp, P(PlanInfo)]),
        "obfft_workspace_size": (ctypes.c_size_t, [vp]),
        "obfft_set_workspace": (i32, [vp, vp, ctypes.c_size_t]),
        "obfft_plan_roots": (i32, [vp, i32, P(i64)]),
        "fft3d_z2z_forward": (i32, [vp, vp, vp, vp]),
        "fft3d_z2z_forward_noalloc": (i32, [vp, vp, vp, vp]),
        "obfft_noalloc_scratch_bytes": (ctypes.c_size_t, []),
        "fft3d_z2z_inverse": (i32, [vp, vp, vp, vp]),
        "fft3d_z2z_adjoint": (i32, [vp, vp, vp, vp]),
        "fft3d_c2c_forward": (i32, [vp, vp, vp, vp]),
        "fft3d_c2c_inverse": (i32, [vp, vp, vp, vp]),
        "fft3d_z2z_native_forward": (i32, [vp, vp, vp, vp]),
        "fft3d_z2z_native_inverse": (i32, [vp, vp, vp, vp]),
        "obfft_stage": (i32, [vp, i32, i32, i32, vp, vp, vp, vp]),
        "obfft_debug_tap": (i32, [vp, i32, i32, i32, i64, vp, vp, vp, vp]),
        "obfft_crt_reconstruct": (i32, [i32, i64, vp, vp, vp, vp, vp]),
        "obfft_crt_reconstruct_method": (i32, [i32, i32, i64, vp, vp, vp, vp]),
        "obfft_taps_layout": (None, [P(TapsLayout)]),
        "obfft_mfma_probe": (i32, [i32, vp, vp, vp, vp]),
        "obfft_quantised_roots": (i32, [i64, i32, P(i64)]),
        "obfft_crt_constants": (i32, [i32, P(CrtConstants)]),
        "obfft_batch_plan_create": (i32, [P(vp), i32, P(i64), P(Options)]),
        "obfft_batch_plan_create_each": (i32, [P(vp), i32, P(i64), P(Options)]),
        "obfft_batch_forward": (i32, [vp, P(vp), P(vp), vp]),
        "obfft_batch_set_graph": (i32, [vp, i32]),
        "obfft_batch_set_mode": (i32, [vp, i32]),
        "obfft_batch_set_poll_limit": (i32, [vp, i32]),
        "obfft_batch_set_claim": (i32, [vp, i32]),
        "obfft_batch_get_claim": (i32, [vp]),
        "obfft_status_string": (ctypes.c_char_p, [i32]),
        "obfft_last_error": (i32, [vp]),
        "obfft_clear_error": (i32, [vp]),
    }
    for name, (res, args) in sigs.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def status_string(s):
    try:
        return lib().obfft_status_string(int(s)).decode()
    except ImportError:
        return f"status {s}"


def check(status, what=""):
    if status != 0:
        raise ObfftError(status, what)


EXPORTED = ["obfft_options_default", "obfft_plan_create", "obfft_plan_destroy", "obfft_plan_info",
            "obfft_workspace_size", "obfft_set_workspace", "obfft_plan_roots", "fft3d_z2z_forward",
            "fft3d_z2z_inverse", "fft3d_z2z_adjoint", "fft3d_c2c_forward", "fft3d_c2c_inverse",
            "fft3d_z2z_native_forward", "fft3d_z2z_native_inverse", "obfft_stage", "obfft_debug_tap",
            "obfft_crt_reconstruct", "obfft_crt_reconstruct_method", "obfft_taps_layout", "obfft_mfma_probe",
            "obfft_quantised_roots", "obfft_crt_constants", "obfft_batch_plan_create",
            "obfft_batch_forward", "obfft_batch_set_graph", "obfft_batch_set_mode", "obfft_batch_set_poll_limit",
            "obfft_status_string", "obfft_last_error",
            "obfft_clear_error", "fft3d_z2z_forward_noalloc", "obfft_noalloc_scratch_bytes",
            "obfft_batch_plan_create_each", "obfft_batch_set_claim", "obfft_batch_get_claim"]
