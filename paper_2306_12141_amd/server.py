"""Serving loop over resident content (include/recoil_server.h): argument marshalling only."""

from __future__ import annotations

import ctypes as C
from typing import List, Optional

import numpy as np

from . import _lib
from ._lib import Completion, ServerConfig, ServerStats, Tuning, check


def now_ns() -> int:
    return int(_lib.recoil_server_now_ns())


class Server:
    """Requests for resident blobs, decoded by continuous batching on the GPU.

    `arena` is a caller-owned uint8 device tensor; its first `resident_bytes`
    hold the content, the rest (minus small per-stream control regions) is the
    request budget.
    """

    def __init__(self, arena, resident_bytes: int, hip_streams: int = 2, max_batch: int = 256,
                 prep_threads: int = 4, items_per_launch: int = 1 << 17, tuning: Optional[Tuning] = None,
                 long_unit_bytes: int = 0, long_streams: int = 0):
        self.arena = arena
        cfg = ServerConfig(hip_streams, max_batch, prep_threads, items_per_launch, resident_bytes,
                           tuning if tuning is not None else _lib.recoil_default_tuning(), long_unit_bytes,
                           long_streams, 0)
        self._h = C.c_void_p()
        check(_lib.recoil_server_create(C.byref(cfg), C.c_void_p(arena.data_ptr()), arena.numel(),
                                        C.byref(self._h)), "recoil_server_create")
        self._contents = []
        self._buf = (Completion * 4096)()

    def close(self) -> None:
        h = getattr(self, "_h", None)
        if h:
            _lib.recoil_server_destroy(h)
            self._h = None

    def __del__(self, _destroy=_lib.recoil_server_destroy):
        h = getattr(self, "_h", None)
        if h:
            _destroy(h)
            self._h = None

    def add_content(self, blob) -> int:
        cid = C.c_uint32()
        check(_lib.recoil_server_add_content(self._h, blob.handle, C.byref(cid)), "recoil_server_add_content")
        self._contents.append(blob)
        return cid.value

    def submit(self, content: int, splits: int = 0, tag: int = 0, arrival_ns: int = 0) -> int:
        rid = C.c_uint64()
        check(_lib.recoil_server_submit(self._h, content, splits, tag, arrival_ns, C.byref(rid)),
              "recoil_server_submit")
        return rid.value

    def poll(self, timeout_us: int = 0, cap: int = 4096) -> List[Completion]:
        n = _lib.recoil_server_poll(self._h, self._buf, min(cap, len(self._buf)), timeout_us)
        return [Completion.from_buffer_copy(self._buf[i]) for i in range(n)]

    def release(self, request_id: int) -> None:
        check(_lib.recoil_server_release(self._h, request_id), "recoil_server_release")

    def stats(self) -> ServerStats:
        st = ServerStats()
        check(_lib.recoil_server_get_stats(self._h, C.byref(st)), "recoil_server_get_stats")
        return st

    def output_of(self, c: Completion, dtype) -> np.ndarray:
        """Host copy of a completed request's symbols (before it is released)."""
        host = self.arena[c.out_offset: c.out_offset + c.out_bytes].cpu().numpy()
        return host.view(dtype)
