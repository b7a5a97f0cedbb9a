"""Batched decoding of many Recoil streams in one persistent launch (include/recoil_batch.h)."""

from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np

from . import _lib
from ._lib import Tuning, check


def _stream_handle(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    if hasattr(stream, "cuda_stream"):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


def default_tuning() -> Tuning:
    return _lib.recoil_default_tuning()


class Batch:
    """A set of blobs decoded together; owns nothing on the device."""

    def __init__(self, blobs: Sequence, tuning: Optional[Tuning] = None):
        self._blobs = list(blobs)          # keep the Python handles alive
        arr = (C.c_void_p * len(self._blobs))(*[b.handle.value for b in self._blobs])
        self._h = C.c_void_p()
        ws, ob = C.c_size_t(), C.c_size_t()
        check(_lib.recoil_batch_create(C.cast(arr, C.c_void_p), len(self._blobs),
                                       C.byref(tuning) if tuning is not None else None, C.byref(self._h),
                                       C.byref(ws), C.byref(ob)), "recoil_batch_create")
        self.workspace_bytes = ws.value
        self.output_bytes = ob.value
        self.count = len(self._blobs)

    def __del__(self, _free=_lib.recoil_batch_free):
        h = getattr(self, "_h", None)
        if h:
            _free(h)
            self._h = None

    @property
    def items(self) -> int:
        return _lib.recoil_batch_items(self._h)

    def output_range(self, i: int):
        off, n = C.c_uint64(), C.c_uint64()
        check(_lib.recoil_batch_output_offset(self._h, i, C.byref(off), C.byref(n)), "recoil_batch_output_offset")
        return off.value, n.value

    def allocate(self, device="cuda"):
        import torch
        ws = torch.empty(max(self.workspace_bytes, 256), dtype=torch.uint8, device=device)
        out = torch.empty(max(self.output_bytes, 256), dtype=torch.uint8, device=device)
        err = torch.zeros(1, dtype=torch.int32, device=device)
        return ws, out, err

    def upload(self, ws, stream=None):
        check(_lib.recoil_batch_upload(self._h, C.c_void_p(ws.data_ptr()), ws.numel(), _stream_handle(stream)),
              "recoil_batch_upload")

    @property
    def tuning(self) -> Tuning:
        t = Tuning()
        check(_lib.recoil_batch_get_tuning(self._h, C.byref(t)), "recoil_batch_get_tuning")
        return t

    def set_tuning(self, t: Tuning, ws=None, stream=None):
        check(_lib.recoil_batch_set_tuning(self._h, C.byref(t), C.c_void_p(ws.data_ptr()) if ws is not None else None,
                                           _stream_handle(stream)), "recoil_batch_set_tuning")

    def decode(self, ws, out, err, stream=None):
        check(_lib.recoil_decode_batch(self._h, C.c_void_p(ws.data_ptr()), C.c_void_p(out.data_ptr()),
                                       C.c_void_p(err.data_ptr()), _stream_handle(stream)), "recoil_decode_batch")

    def decode_noalloc(self, ws, out, err, stream=None):
        """recoil_decode_batch_noalloc: queue heads in the library's static device array."""
        check(_lib.recoil_decode_batch_noalloc(self._h, C.c_void_p(ws.data_ptr()), C.c_void_p(out.data_ptr()),
                                               C.c_void_p(err.data_ptr()), _stream_handle(stream)),
              "recoil_decode_batch_noalloc")

    def decode_per_stream(self, ws, out, err, stream=None):
        check(_lib.recoil_decode_batch_per_stream(self._h, C.c_void_p(ws.data_ptr()), C.c_void_p(out.data_ptr()),
                                                  C.c_void_p(err.data_ptr()), _stream_handle(stream)),
              "recoil_decode_batch_per_stream")

    def graph(self, ws, out, err) -> "Graph":
        g = C.c_void_p()
        check(_lib.recoil_batch_graph_create(self._h, C.c_void_p(ws.data_ptr()), C.c_void_p(out.data_ptr()),
                                             C.c_void_p(err.data_ptr()), C.byref(g)), "recoil_batch_graph_create")
        return Graph(g)

    def autotune(self, ws, out, err, reps: int = 3, stream=None):
        best = Tuning()
        ms = C.c_float()
        check(_lib.recoil_autotune(self._h, C.c_void_p(ws.data_ptr()), C.c_void_p(out.data_ptr()),
                                   C.c_void_p(err.data_ptr()), _stream_handle(stream), reps, C.byref(best),
                                   C.byref(ms)), "recoil_autotune")
        return best, ms.value

    def symbols_of(self, out, i: int, dtype) -> np.ndarray:
        off, n = self.output_range(i)
        return out[off:off + n].cpu().numpy().view(dtype)


class Graph:
    """An instantiated HIP graph of [queue reset; persistent batched decode]."""

    def __init__(self, handle):
        self._h = handle

    def __del__(self, _free=_lib.recoil_graph_free):
        h = getattr(self, "_h", None)
        if h:
            _free(h)
            self._h = None

    def launch(self, stream=None):
        check(_lib.recoil_graph_launch(self._h, _stream_handle(stream)), "recoil_graph_launch")
