"""ctypes declarations of libboa's C ABI (include/boa.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# BOA_LIB_PATH selects another build of the same library (the host-sanitizer
# build of paper_2511_11337_amd.sanitize)
LIB_PATH = os.environ.get("BOA_LIB_PATH") or os.path.join(_HERE, "libboa.so")

BOA_OK = 0
ERRORS = {
    -1: "BOA_E_ARG", -2: "BOA_E_OOM", -3: "BOA_E_DEVICE", -4: "BOA_E_FORMAT",
    -5: "BOA_E_CRC", -6: "BOA_E_MODEL", -7: "BOA_E_CORRUPT", -8: "BOA_E_UNSUPPORTED",
}
DTYPES = {"f32": 0, "fp32": 0, "float32": 0, "bf16": 1, "bfloat16": 1, "fp8": 2, "int8": 3}


class BoaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


class boa_config(C.Structure):
    _fields_ = [("d_model", C.c_uint32), ("n_layers", C.c_uint32), ("d_state", C.c_uint32),
                ("d_conv", C.c_uint32), ("expand", C.c_uint32), ("ffn_mult", C.c_uint32)]


class boa_run_opts(C.Structure):
    _fields_ = [("dtype", C.c_uint32), ("max_lanes", C.c_uint32), ("tile_t", C.c_uint32),
                ("use_graph", C.c_uint32), ("fallback", C.c_uint32), ("decode_groups", C.c_uint32),
                ("decode_kernel", C.c_uint32), ("fused_lanes", C.c_uint32)]


class boa_train_opts(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("weight_decay", C.c_float), ("grad_clip", C.c_float), ("warmup", C.c_uint32),
                ("steps", C.c_uint32), ("batch", C.c_uint32), ("seq_len", C.c_uint32),
                ("chunk_t", C.c_uint32), ("dtype", C.c_uint32), ("seed", C.c_uint64)]


P = C.c_void_p
U64P = C.POINTER(C.c_uint64)
U32 = C.c_uint32
U64 = C.c_uint64

# name -> (restype, argtypes); every symbol include/boa.h declares
SIGNATURES = {
    "boa_param_count": (U64, [C.POINTER(boa_config)]),
    "boa_model_create": (C.c_int, [C.POINTER(boa_config), P, U64, C.c_int, C.POINTER(P)]),
    "boa_model_free": (None, [P]),
    "boa_model_get_weights": (C.c_int, [P, P, U64]),
    "boa_model_set_weights": (C.c_int, [P, P, U64]),
    "boa_model_config": (C.c_int, [P, C.POINTER(boa_config)]),
    "boa_model_fingerprint": (C.c_int, [P, U64P]),
    "boa_model_save": (C.c_int, [P, C.c_char_p]),
    "boa_model_load": (C.c_int, [C.c_char_p, C.c_int, C.POINTER(P)]),
    "boa_compress": (C.c_int, [P, P, U64P, U64, C.POINTER(boa_run_opts), C.POINTER(P), U64P]),
    "boa_decompress": (C.c_int, [P, P, U64, C.POINTER(boa_run_opts), C.POINTER(P), U64P]),
    "boa_container_info": (C.c_int, [P, U64, U64P, U64P, U64P, C.POINTER(U32)]),
    "boa_last_chunk_stats": (C.c_int, [U64P, C.POINTER(U32), U64]),
    "boa_free": (None, [P]),
    "boa_last_error": (C.c_char_p, []),
    "boa_numerics_id": (U32, [U32]),
    "boa_workspace_size": (C.c_int, [P, U64P, U64, C.POINTER(boa_run_opts), U32, U64P]),
    "boa_split_fixed": (C.c_int, [U64, U64, U64P, U64, U64P]),
    "boa_plan_lanes": (C.c_int, [U64P, U64, C.c_uint32, C.POINTER(C.c_uint32)]),
    "boa_payload_layout": (C.c_int, [U64P, U64, U64P, U64P, U64P, U64P]),
    "boa_encode_dev": (C.c_int, [P, P, U64P, U64P, U64, C.POINTER(boa_run_opts), P, U64P, U64P, P, P, P, U64, P]),
    "boa_decode_dev": (C.c_int, [P, P, U64P, U64P, P, U64P, U64P, U64, C.POINTER(boa_run_opts), P, P, U64, P]),
    "boa_decode_noalloc_dev": (C.c_int, [P, P, U64P, U64P, P, U64P, U64P, U64, C.POINTER(boa_run_opts), P, P]),
    "boa_logits_dev": (C.c_int, [P, P, U32, U32, U32, U32, P, P, P, P]),
    "boa_diagnostics_dev": (C.c_int, [P, P, U32, U32, U32, U32, U32, P, P, P, P]),
    "boa_diagnostics_summary": (C.c_int, [P, P, U32, P, P, U64P]),
    "boa_stream_open": (C.c_int, [P, U64, U32, U32, P, P]),
    "boa_stream_push": (C.c_int, [P, P, U64]),
    "boa_stream_finish": (C.c_int, [P]),
    "boa_stream_next_shard": (C.c_int, [P, C.c_int, P, P]),
    "boa_stream_close": (None, [P]),
    "boa_code_tables_dev": (C.c_int, [P, P, U64P, U64, P, U64P, U64P, P, P]),
    "boa_decode_tables_dev": (C.c_int, [P, U64P, U64P, P, U64P, U64, P, P]),
    "boa_order2_encode_dev": (C.c_int, [P, U64P, U64P, U64, P, U64P, U64P, P, P, P]),
    "boa_order2_decode_dev": (C.c_int, [P, U64P, U64P, P, U64P, U64P, U64, P, P]),
    "boa_prof_enable": (C.c_int, [U32]),
    "boa_prof_read": (C.c_int, [P, P, C.c_int]),
    "boa_loss_grad_dev": (C.c_int, [P, P, U32, U32, U32, U32, P, P, P]),
    "boa_optimizer_step_dev": (C.c_int, [P, P, C.POINTER(boa_train_opts), P]),
    "boa_train_step_dev": (C.c_int, [P, P, U32, U32, C.POINTER(boa_train_opts), P, P]),
    "boa_train_state_save": (C.c_int, [P, C.c_char_p]),
    "boa_train_state_load": (C.c_int, [P, C.c_char_p]),
    "boa_train_steps_done": (C.c_int, [P, U64P]),
    "boa_train": (C.c_int, [P, P, U64, C.POINTER(boa_train_opts), P, U64]),
    "boa_scan_fwd_dev": (C.c_int, [P, P, P, P, P, U32, U32, U32, U32, P, P, P]),
    "boa_scan_bwd_dev": (C.c_int, [P, P, P, P, P, P, U32, U32, U32, U32, P, P, P, P, P, P, P]),
    "boa_qmodel_create": (C.c_int, [P, C.POINTER(P)]),
    "boa_qmodel_free": (None, [P]),
    "boa_int_tables_dev": (C.c_int, [P, P, U32, U32, P, P, P]),
    "boa_int_encode_dev": (C.c_int, [P, P, U64P, U64P, U64, P, U64P, U64P, P, P]),
    "boa_int_decode_dev": (C.c_int, [P, P, U64P, U64P, P, U64P, U64P, U64, P, P]),
}

_lib = None


def load() -> C.CDLL:
    """Load the in-tree libboa.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libboa.so not built at {LIB_PATH}; run `python -m paper_2511_11337_amd.build`")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(rc: int) -> None:
    if rc != BOA_OK:
        msg = load().boa_last_error()
        raise BoaError(rc, msg.decode() if msg else "")


def u64_array(values):
    arr = (C.c_uint64 * len(values))(*[int(v) for v in values])
    return arr
