"""ctypes binding of librecoil.so (argument marshalling only).

Every decode step runs in the library's HIP kernels; this module converts
numpy arrays and torch tensors into plain pointers and sizes. It raises at
import time if the built library is missing: there is no fallback path.
"""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(HERE, "librecoil.so")

if not os.path.exists(SO_PATH):
    raise ImportError(
        f"librecoil.so not found at {SO_PATH}; build it with `python -m paper_2306_12141_amd.build` "
        "(hipcc, gfx950). There is no CPU fallback.")

lib = C.CDLL(SO_PATH)

P = C.c_void_p
u32 = C.c_uint32
u64 = C.c_uint64
i32 = C.c_int32
sz = C.c_size_t


class Config(C.Structure):
    _fields_ = [("lanes", u32), ("quant_bits", u32), ("symbol_bytes", u32), ("alphabet", u32)]


class BlobInfo(C.Structure):
    _fields_ = [("n_symbols", u64), ("n_words", u64), ("splits", u32), ("lanes", u32),
                ("quant_bits", u32), ("symbol_bytes", u32), ("alphabet", u32),
                ("table_bytes", u64), ("metadata_bytes", u64), ("total_bytes", u64)]


def _sig(name, args, res=i32):
    fn = getattr(lib, name)
    fn.argtypes = args
    fn.restype = res
    return fn


recoil_status_string = _sig("recoil_status_string", [i32], C.c_char_p)
recoil_last_error = _sig("recoil_last_error", [], C.c_char_p)
recoil_version = _sig("recoil_version", [], C.c_char_p)
recoil_quantize = _sig("recoil_quantize", [P, u32, u32, P])
recoil_encode = _sig("recoil_encode", [P, u64, C.POINTER(Config), P, u32, C.POINTER(P)])
recoil_encode_adaptive = _sig("recoil_encode_adaptive", [P, u64, C.POINTER(Config), P, u32, P, u32, C.POINTER(P)])
recoil_decode_adaptive = _sig("recoil_decode_adaptive", [P, P, P, P, P, P])
recoil_encode_partitioned = _sig("recoil_encode_partitioned", [P, u64, C.POINTER(Config), P, u32, C.POINTER(P)])
recoil_combine_splits = _sig("recoil_combine_splits", [P, u32, C.POINTER(P)])
recoil_set_split_writer_threads = _sig("recoil_set_split_writer_threads", [u32], None)
recoil_blob_serialize = _sig("recoil_blob_serialize", [P, P, sz, C.POINTER(sz)])
recoil_blob_deserialize = _sig("recoil_blob_deserialize", [P, sz, C.POINTER(P)])
recoil_blob_info = _sig("recoil_blob_info", [P, C.POINTER(BlobInfo)])
recoil_blob_free = _sig("recoil_blob_free", [P], None)
recoil_plan_create = _sig("recoil_plan_create", [P, C.POINTER(P), C.POINTER(sz)])
recoil_plan_upload = _sig("recoil_plan_upload", [P, P, sz, P])
recoil_plan_metadata_device_bytes = _sig("recoil_plan_metadata_device_bytes", [P], sz)
recoil_plan_free = _sig("recoil_plan_free", [P], None)
recoil_decode = _sig("recoil_decode", [P, P, P, P, P])
recoil_decode_count_writes = _sig("recoil_decode_count_writes", [P, P, P, P, P, P])
recoil_plan_units = _sig("recoil_plan_units", [P, P, u32, C.POINTER(u32)])
recoil_plan_create_packed = _sig("recoil_plan_create_packed", [P, u32, C.POINTER(P), C.POINTER(sz)])
recoil_plan_unpack = _sig("recoil_plan_unpack", [P, P, P])


class PlanLayout(C.Structure):
    _fields_ = [("words", sz), ("table", sz), ("units", sz), ("lanes", sz), ("total", sz),
                ("unit_count", u32), ("lanes_per_unit", u32), ("packed", u32)]


recoil_plan_get_layout = _sig("recoil_plan_get_layout", [P, C.POINTER(PlanLayout)])
recoil_plan_decode_table = _sig("recoil_plan_decode_table", [P, P, sz, C.POINTER(sz)])


class RecoilError(RuntimeError):
    def __init__(self, status: int, what: str):
        msg = recoil_last_error().decode(errors="replace")
        super().__init__(f"{what}: {recoil_status_string(status).decode()} ({status}): {msg}")
        self.status = status


def check(status: int, what: str) -> None:
    if status != 0:
        raise RecoilError(status, what)


class Tuning(C.Structure):
    _fields_ = [("waves", u32), ("chunk_groups", u32), ("pairs_per_wave", u32), ("blocks_per_cu", u32),
                ("units_per_run", u32)]


class DecodeShape(C.Structure):
    _fields_ = [("blocks", u32), ("waves_per_block", u32), ("units_per_run", u32), ("runs", u32),
                ("units_per_wave", u32)]


recoil_plan_set_tuning = _sig("recoil_plan_set_tuning", [P, C.POINTER(Tuning)])
recoil_plan_shape = _sig("recoil_plan_shape", [P, C.POINTER(DecodeShape)])
recoil_plan_autotune = _sig("recoil_plan_autotune", [P, P, P, P, P, u32, C.POINTER(Tuning), C.POINTER(C.c_float)])
recoil_default_tuning = _sig("recoil_default_tuning", [], Tuning)
recoil_batch_create = _sig("recoil_batch_create", [P, u32, C.POINTER(Tuning), C.POINTER(P), C.POINTER(sz),
                                                   C.POINTER(sz)])
recoil_batch_free = _sig("recoil_batch_free", [P], None)
recoil_batch_output_offset = _sig("recoil_batch_output_offset", [P, u32, C.POINTER(u64), C.POINTER(u64)])
recoil_batch_items = _sig("recoil_batch_items", [P], u32)
recoil_batch_upload = _sig("recoil_batch_upload", [P, P, sz, P])
recoil_batch_set_tuning = _sig("recoil_batch_set_tuning", [P, C.POINTER(Tuning), P, P])
recoil_batch_get_tuning = _sig("recoil_batch_get_tuning", [P, C.POINTER(Tuning)])
recoil_decode_batch = _sig("recoil_decode_batch", [P, P, P, P, P])
recoil_decode_batch_noalloc = _sig("recoil_decode_batch_noalloc", [P, P, P, P, P])
recoil_decode_batch_per_stream = _sig("recoil_decode_batch_per_stream", [P, P, P, P, P])
recoil_batch_graph_create = _sig("recoil_batch_graph_create", [P, P, P, P, C.POINTER(P)])
recoil_graph_launch = _sig("recoil_graph_launch", [P, P])
recoil_graph_free = _sig("recoil_graph_free", [P], None)
recoil_autotune = _sig("recoil_autotune", [P, P, P, P, P, u32, C.POINTER(Tuning), C.POINTER(C.c_float)])


class ServerConfig(C.Structure):
    _fields_ = [("hip_streams", u32), ("max_batch", u32), ("prep_threads", u32), ("items_per_launch", u32),
                ("resident_bytes", u64), ("tuning", Tuning), ("long_unit_bytes", u64), ("long_streams", u32),
                ("reserved", u32)]


class Completion(C.Structure):
    _fields_ = [("request_id", u64), ("tag", u64), ("content", u32), ("splits", u32), ("status", i32),
                ("device_error", u32), ("out_offset", u64), ("out_bytes", u64), ("metadata_bytes", u64),
                ("t_arrival_ns", u64), ("t_admit_ns", u64), ("t_launch_ns", u64), ("t_done_ns", u64)]


class ServerStats(C.Structure):
    _fields_ = [(n, u64) for n in ("submitted", "completed", "rejected", "launches", "requests_launched",
                                   "pending", "in_flight", "budget_bytes", "budget_used", "budget_peak",
                                   "resident_used", "decoded_bytes")]


recoil_server_now_ns = _sig("recoil_server_now_ns", [], u64)
recoil_server_create = _sig("recoil_server_create", [C.POINTER(ServerConfig), P, sz, C.POINTER(P)])
recoil_server_add_content = _sig("recoil_server_add_content", [P, P, C.POINTER(u32)])
recoil_server_submit = _sig("recoil_server_submit", [P, u32, u32, u64, u64, C.POINTER(u64)])
recoil_server_poll = _sig("recoil_server_poll", [P, C.POINTER(Completion), u32, u32], u32)
recoil_server_release = _sig("recoil_server_release", [P, u64])
recoil_server_get_stats = _sig("recoil_server_get_stats", [P, C.POINTER(ServerStats)])
recoil_server_destroy = _sig("recoil_server_destroy", [P], None)
