"""ctypes declarations of the libcompar C ABI (include/compar.h).

Only argument marshalling lives here: every computation runs inside
libcompar.so (host runtime + gfx950 kernels).  Loading fails loudly when the
library has not been built; nothing falls back to Python or the CPU.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# COMPAR_SANITIZED=1 loads the host-sanitized build (build.py, sanitize=True) instead
LIB_PATH = os.path.join(HERE, "libcompar_san.so" if os.environ.get("COMPAR_SANITIZED") == "1" else "libcompar.so")

# status codes (cmp_status)
CMP_OK = 0
CMP_EINVAL = -1
CMP_EDUP = -2
CMP_ESIG = -3
CMP_ENOTFOUND = -4
CMP_ENOVARIANT = -5
CMP_EUNSUPPORTED = -6
CMP_EHIP = -7
CMP_ENOMEM = -8
CMP_ECHECK = -9
CMP_ENODATA = -10

CMP_TARGET_HIP = 1
CMP_TARGET_HOST = 2
CMP_F32, CMP_BF16, CMP_F8E4M3, CMP_F64, CMP_I32, CMP_I64 = range(6)
CMP_READ, CMP_WRITE, CMP_READWRITE = 1, 2, 3
CMP_SEL_STATIC, CMP_SEL_NN, CMP_SEL_MLP = 0, 1, 2
CMP_FLAG_VERIFY = 1
CMP_FLAG_LOG = 2


class cmp_param_desc(C.Structure):
    _fields_ = [("name", C.c_char_p), ("type", C.c_int32), ("ndim", C.c_int32),
                ("extent", C.c_char_p * 4), ("mode", C.c_int32)]


class cmp_gemm_args(C.Structure):
    _fields_ = [("M", C.c_int64), ("N", C.c_int64), ("K", C.c_int64),
                ("lda", C.c_int64), ("ldb", C.c_int64), ("ldc", C.c_int64),
                ("alpha", C.c_float), ("beta", C.c_float),
                ("A", C.c_void_p), ("B", C.c_void_p), ("C", C.c_void_p)]


class cmp_image_layout(C.Structure):
    _fields_ = [("Mp", C.c_int64), ("Np", C.c_int64), ("Kp", C.c_int64), ("count", C.c_int32),
                ("offset", C.c_int64 * 8), ("bytes", C.c_int64 * 8), ("total", C.c_int64)]


class cmp_context(C.Structure):
    _fields_ = [("M", C.c_int64), ("N", C.c_int64), ("K", C.c_int64),
                ("dtype", C.c_int32), ("tol", C.c_double)]


cmp_variant_fn = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
cmp_ws_fn = C.CFUNCTYPE(C.c_size_t, C.c_void_p, C.c_void_p)

_P = C.c_void_p
_I = C.c_int
_I64 = C.c_int64
_U64 = C.c_uint64
_F = C.c_float
_D = C.c_double
_S = C.c_char_p
_FP = C.POINTER(C.c_float)
_DP = C.POINTER(C.c_double)
_IP = C.POINTER(C.c_int)

# name -> (restype, argtypes); the exported symbol set of include/compar.h
SIGNATURES = {
    "cmp_init": (_I, [_I, C.POINTER(_P)]),
    "cmp_terminate": (_I, [_P]),
    "cmp_last_error": (_S, [_P]),
    "cmp_status_string": (_S, [_I]),
    "cmp_version": (_S, []),
    "cmp_device": (_I, [_P, _IP, C.c_char_p, C.c_size_t, _IP, _IP]),
    "cmp_interface_declare": (_I, [_P, _S, _I, C.POINTER(cmp_param_desc)]),
    "cmp_variant_register": (_I, [_P, _S, _S, _I, _I, C.POINTER(cmp_param_desc), cmp_variant_fn,
                                  cmp_ws_fn, _D, _P, _IP]),
    "cmp_variant_count": (_I, [_P, _S, _IP]),
    "cmp_variant_info": (_I, [_P, _S, _I, C.POINTER(_S), _IP, _DP]),
    "cmp_variant_find": (_I, [_P, _S, _S, _IP]),
    "cmp_set_variant_mask": (_I, [_P, _S, _U64]),
    "cmp_force_variant": (_I, [_P, _S, _I]),
    "cmp_selector_set": (_I, [_P, _I]),
    "cmp_set_flags": (_I, [_P, C.c_uint32]),
    "cmp_set_log_file": (_I, [_P, C.c_char_p]),
    "cmp_reserve": (_I, [_P, C.c_int64, C.c_int64, C.c_int64]),
    "cmp_log_flush": (_I, [_P]),
    "cmp_set_split_k": (_I, [_P, _I]),
    "cmp_register_builtin": (_I, [_P, _S, _IP]),
    "cmp_quant_mx6": (_I, [_P, _I64, _I64, _P, _I64, _I, _P, _P, _P, _P, _P]),
    "cmp_split_k": (_I, [_P, _I, C.c_int64, C.c_int64, C.c_int64, _IP]),
    "cmp_admissible": (_I, [_P, _S, C.POINTER(cmp_context), C.POINTER(_U64)]),
    "cmp_select": (_I, [_P, _S, C.POINTER(cmp_context), _IP]),
    "cmp_select_batch": (_I, [_P, _S, _I, C.POINTER(cmp_context), _IP]),
    "cmp_gemm": (_I, [_P, C.POINTER(cmp_gemm_args), _D, _P, _IP]),
    "cmp_gemm_stream": (_I, [_P, _I, C.POINTER(cmp_gemm_args), _DP, C.POINTER(C.c_uint32), _I, _P, _IP,
                             _DP, _IP]),
    "cmp_gemm_variant": (_I, [_P, _I, C.POINTER(cmp_gemm_args), _P]),
    "cmp_gemm_variant_static": (_I, [_P, _I, C.POINTER(cmp_gemm_args), _P]),
    "cmp_call_host": (_I, [_P, _S, _I, _P]),
    "cmp_time_variant": (_I, [_P, _I, C.POINTER(cmp_gemm_args), _I, _I, _P, _FP, _FP, _FP]),
    "cmp_calibrate": (_I, [_P, _I, C.POINTER(C.c_int64), _P, _P, _P, _I, _I, _P]),
    "cmp_history_add": (_I, [_P, _I64, _I64, _I64, _I, _I, _F, _F, _F]),
    "cmp_history_count": (_I, [_P, _IP]),
    "cmp_history_get": (_I, [_P, _I, C.POINTER(C.c_int64), _IP, _IP, _FP, _FP, _FP]),
    "cmp_history_clear": (_I, [_P]),
    "cmp_history_save": (_I, [_P, _S]),
    "cmp_history_load": (_I, [_P, _S, _I]),
    "cmp_mlp_param_count": (_I, []),
    "cmp_mlp_set_params": (_I, [_P, _FP, _I]),
    "cmp_mlp_get_params": (_I, [_P, _FP, _I]),
    "cmp_mlp_set_norm": (_I, [_P, _FP, _FP, _FP, _FP]),
    "cmp_mlp_get_norm": (_I, [_P, _FP, _FP, _FP, _FP]),
    "cmp_mlp_train": (_I, [_P, _I, _FP, _FP, _I, _F, _FP]),
    "cmp_mlp_grad": (_I, [_P, _I, _FP, _FP, _FP, _FP]),
    "cmp_mlp_infer": (_I, [_P, _I, _FP, _FP]),
    "cmp_mlp_fit_history": (_I, [_P, _I, _F, _U64, _FP]),
    "cmp_mlp_save": (_I, [_P, C.c_char_p]),
    "cmp_mlp_load": (_I, [_P, C.c_char_p, _I]),
    "cmp_freivalds": (_I, [_P, C.POINTER(cmp_gemm_args), _P, _DP, _P, _DP]),
    "cmp_last_verify": (_I, [_P, _DP, _IP]),
    "cmp_split_bf16": (_I, [_P, _I64, _I64, _P, _I64, _P, _P, _P]),
    "cmp_quant_fp8": (_I, [_P, _I64, _I64, _P, _I64, _P, _P, _P, _P, _P]),
    "cmp_prepass_layout": (_I, [_P, _I, _I64, _I64, _I64, C.POINTER(cmp_image_layout)]),
    "cmp_prepass_images": (_I, [_P, _I, C.POINTER(cmp_gemm_args), _P, C.c_size_t, _P]),
    "cmp_grouped_config_count": (_I, []),
    "cmp_grouped_config_info": (_I, [_I, _IP, _IP, _IP]),
    "cmp_grouped_config_variant": (_I, [_I, _IP]),
    "cmp_grouped_plan_create": (_I, [_P, _I, C.POINTER(cmp_gemm_args), _I, _I, _P, C.POINTER(_P)]),
    "cmp_grouped_plan_info": (_I, [_P, _IP, _IP, _IP, _IP, _FP]),
    "cmp_grouped_launch": (_I, [_P, _P]),
    "cmp_grouped_graph_launch": (_I, [_P, _P]),
    "cmp_grouped_plan_destroy": (_I, [_P]),
    "cmp_kernel_timing": (_I, [_P, _I]),
    "cmp_kernel_stats": (_I, [_P, _I, C.c_char_p, C.c_size_t, C.POINTER(C.c_longlong), _DP]),
}

_lib = None


def load():
    """Load libcompar.so and declare every entry point; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "or python paper_2311_03543_amd/build.py")
    L = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


class ComparError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{status_name(status)}: {message}")
        self.status = status


def status_name(st: int) -> str:
    return load().cmp_status_string(st).decode()
