"""librecoil: Recoil parallel rANS decoding on AMD MI355X (gfx950).

Python surface over the C-ABI in include/recoil.h. Host arrays are numpy;
device buffers are torch tensors on a ROCm device (used only for their memory
and streams). Every decode runs in the HIP kernels of librecoil.so.
"""

from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np

from . import _lib
from ._lib import RecoilError, check

__all__ = ["Blob", "Plan", "encode", "quantize", "RecoilError", "version"]


def version() -> str:
    return _lib.recoil_version().decode()


def _ptr(a: np.ndarray) -> C.c_void_p:
    return C.c_void_p(a.ctypes.data)


def quantize(counts: np.ndarray, quant_bits: int) -> np.ndarray:
    counts = np.ascontiguousarray(counts, dtype=np.uint64)
    f = np.zeros(len(counts), dtype=np.uint32)
    check(_lib.recoil_quantize(_ptr(counts), len(counts), quant_bits, _ptr(f)), "recoil_quantize")
    return f


class Blob:
    """An encoded stream (bitstream + split metadata); immutable."""

    def __init__(self, handle: C.c_void_p):
        self._h = handle

    def __del__(self, _free=_lib.recoil_blob_free):
        h = getattr(self, "_h", None)
        if h:
            _free(h)
            self._h = None

    @property
    def handle(self) -> C.c_void_p:
        return self._h

    @property
    def info(self) -> _lib.BlobInfo:
        out = _lib.BlobInfo()
        check(_lib.recoil_blob_info(self._h, C.byref(out)), "recoil_blob_info")
        return out

    @property
    def splits(self) -> int:
        return self.info.splits

    @property
    def dtype(self):
        return np.uint8 if self.info.symbol_bytes == 1 else np.uint16

    def combine(self, target_splits: int) -> "Blob":
        h = C.c_void_p()
        check(_lib.recoil_combine_splits(self._h, target_splits, C.byref(h)), "recoil_combine_splits")
        return Blob(h)

    def to_bytes(self) -> bytes:
        n = C.c_size_t()
        check(_lib.recoil_blob_serialize(self._h, None, 0, C.byref(n)), "recoil_blob_serialize")
        buf = np.empty(n.value, dtype=np.uint8)
        check(_lib.recoil_blob_serialize(self._h, _ptr(buf), n.value, C.byref(n)), "recoil_blob_serialize")
        return buf.tobytes()

    @staticmethod
    def from_bytes(data: bytes) -> "Blob":
        buf = np.frombuffer(data, dtype=np.uint8)
        h = C.c_void_p()
        check(_lib.recoil_blob_deserialize(_ptr(buf) if len(buf) else None, len(buf), C.byref(h)),
              "recoil_blob_deserialize")
        return Blob(h)


def set_split_writer_threads(threads: int) -> None:
    """Split selection: 1 streaming (inside the encoder's pass), >= 2 threaded after
    it, 0 automatic (threaded from 2^24 symbols). Same split points either way."""
    _lib.recoil_set_split_writer_threads(int(threads))


def encode(symbols: np.ndarray, lanes: int = 32, quant_bits: int = 11, splits: int = 1,
           alphabet: Optional[int] = None, freq: Optional[np.ndarray] = None) -> Blob:
    """Encode uint8/uint16 symbols into one interleaved stream with `splits` decode units."""
    symbols = np.ascontiguousarray(symbols)
    if symbols.dtype not in (np.uint8, np.uint16):
        raise TypeError("symbols must be uint8 or uint16")
    sb = symbols.dtype.itemsize
    if alphabet is None:
        alphabet = 256 if sb == 1 else 65536
    cfg = _lib.Config(lanes, quant_bits, sb, alphabet)
    fp = None
    if freq is not None:
        freq = np.ascontiguousarray(freq, dtype=np.uint32)
        fp = _ptr(freq)
    h = C.c_void_p()
    check(_lib.recoil_encode(_ptr(symbols) if symbols.size else None, symbols.size, C.byref(cfg), fp,
                             splits, C.byref(h)), "recoil_encode")
    return Blob(h)


def encode_adaptive(symbols: np.ndarray, tables: np.ndarray, table_index: np.ndarray, lanes: int = 32,
                    quant_bits: int = 11, splits: int = 1, alphabet: Optional[int] = None) -> Blob:
    """Adaptive coding (Sec. 3.1): symbol i coded with tables[table_index[i]] (tables: T x A)."""
    symbols = np.ascontiguousarray(symbols)
    if symbols.dtype not in (np.uint8, np.uint16):
        raise TypeError("symbols must be uint8 or uint16")
    tables = np.ascontiguousarray(tables, dtype=np.uint32)
    tidx = np.ascontiguousarray(table_index, dtype=np.uint8)
    if tables.ndim != 2 or len(tidx) != len(symbols):
        raise ValueError("tables must be T x A and table_index one entry per symbol")
    sb = symbols.dtype.itemsize
    if alphabet is None:
        alphabet = tables.shape[1]
    cfg = _lib.Config(lanes, quant_bits, sb, alphabet)
    h = C.c_void_p()
    check(_lib.recoil_encode_adaptive(_ptr(symbols) if symbols.size else None, symbols.size, C.byref(cfg),
                                      _ptr(tables), tables.shape[0], _ptr(tidx) if tidx.size else None, splits,
                                      C.byref(h)), "recoil_encode_adaptive")
    return Blob(h)


def encode_partitioned(symbols: np.ndarray, lanes: int = 32, quant_bits: int = 11, partitions: int = 1,
                       alphabet: Optional[int] = None, freq: Optional[np.ndarray] = None) -> Blob:
    """The conventional baseline (Sec. 2.3): `partitions` independently coded sub-sequences
    (whole groups of `lanes` symbols each) behind an offset table; cannot be combined."""
    symbols = np.ascontiguousarray(symbols)
    if symbols.dtype not in (np.uint8, np.uint16):
        raise TypeError("symbols must be uint8 or uint16")
    sb = symbols.dtype.itemsize
    if alphabet is None:
        alphabet = 256 if sb == 1 else 65536
    cfg = _lib.Config(lanes, quant_bits, sb, alphabet)
    fp = None
    if freq is not None:
        freq = np.ascontiguousarray(freq, dtype=np.uint32)
        fp = _ptr(freq)
    h = C.c_void_p()
    check(_lib.recoil_encode_partitioned(_ptr(symbols) if symbols.size else None, symbols.size, C.byref(cfg), fp,
                                         partitions, C.byref(h)), "recoil_encode_partitioned")
    return Blob(h)


def _stream_handle(stream) -> C.c_void_p:
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    if hasattr(stream, "cuda_stream"):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


class Plan:
    """GPU decode plan of one blob: device workspace layout plus decode launch.

    packed_target=None: records unpacked on the host (recoil_plan_create). An
    integer: recoil_plan_create_packed, the device unpacks the packed metadata
    section at upload, keeping every ceil(M / target)-th split point (0: all)."""

    def __init__(self, blob: Blob, packed_target: Optional[int] = None):
        self._h = C.c_void_p()
        n = C.c_size_t()
        if packed_target is None:
            check(_lib.recoil_plan_create(blob.handle, C.byref(self._h), C.byref(n)), "recoil_plan_create")
        else:
            check(_lib.recoil_plan_create_packed(blob.handle, int(packed_target), C.byref(self._h), C.byref(n)),
                  "recoil_plan_create_packed")
        self.device_bytes = n.value
        info = blob.info
        self.n_symbols = info.n_symbols
        self.symbol_bytes = info.symbol_bytes
        self.splits = info.splits
        self.lanes = info.lanes

    def __del__(self, _free=_lib.recoil_plan_free):
        h = getattr(self, "_h", None)
        if h:
            _free(h)
            self._h = None

    @property
    def metadata_device_bytes(self) -> int:
        return _lib.recoil_plan_metadata_device_bytes(self._h)

    def set_tuning(self, waves: int = 0, chunk_groups: int = 4, blocks_per_cu: int = 0,
                   units_per_run: int = 0) -> None:
        """waves: 1, 8 or 16 per workgroup, or 0 to choose at launch (16, or fewer
        when the decode has too few runs to reach every CU)."""
        t = _lib.Tuning(waves, chunk_groups, 1, blocks_per_cu, units_per_run)
        check(_lib.recoil_plan_set_tuning(self._h, C.byref(t)), "recoil_plan_set_tuning")

    def autotune(self, workspace, out, err, reps: int = 3, stream=None):
        """Time the launch shapes on these buffers and keep the fastest (cached per
        device and stream shape). Returns (tuning, median ms or -1 if cached)."""
        best = _lib.Tuning()
        ms = C.c_float()
        check(_lib.recoil_plan_autotune(self._h, C.c_void_p(workspace.data_ptr()), C.c_void_p(out.data_ptr()),
                                        C.c_void_p(err.data_ptr()), _stream_handle(stream), reps, C.byref(best),
                                        C.byref(ms)), "recoil_plan_autotune")
        return best, ms.value

    def shape(self) -> _lib.DecodeShape:
        """Grid and runs recoil_decode uses for this plan on the current device."""
        sh = _lib.DecodeShape()
        check(_lib.recoil_plan_shape(self._h, C.byref(sh)), "recoil_plan_shape")
        return sh

    def allocate_workspace(self, device="cuda"):
        import torch
        return torch.empty(max(self.device_bytes, 256), dtype=torch.uint8, device=device)

    def upload(self, workspace, stream=None) -> None:
        check(_lib.recoil_plan_upload(self._h, C.c_void_p(workspace.data_ptr()), workspace.numel(),
                                      _stream_handle(stream)), "recoil_plan_upload")

    def unpack(self, workspace, stream=None) -> None:
        """Packed plans: queue the device unpack again on an uploaded workspace."""
        check(_lib.recoil_plan_unpack(self._h, C.c_void_p(workspace.data_ptr()), _stream_handle(stream)),
              "recoil_plan_unpack")

    def allocate_output(self, device="cuda"):
        """A byte tensor of N * symbol_bytes bytes (torch has few uint16 kernels)."""
        import torch
        return torch.empty(max(self.n_symbols * self.symbol_bytes, 16), dtype=torch.uint8, device=device)

    def symbols_of(self, out) -> np.ndarray:
        """Host copy of the decoded symbols held in a byte tensor from allocate_output."""
        host = out[: self.n_symbols * self.symbol_bytes].cpu().numpy()
        return host.view(np.uint8 if self.symbol_bytes == 1 else np.uint16)

    def decode(self, workspace, out, err, stream=None) -> None:
        """Enqueue the decode kernels on `stream` (default: torch's current stream)."""
        if out.numel() * out.element_size() < self.n_symbols * self.symbol_bytes:
            raise ValueError("output tensor too small")
        check(_lib.recoil_decode(self._h, C.c_void_p(workspace.data_ptr()), C.c_void_p(out.data_ptr()),
                                 C.c_void_p(err.data_ptr()), _stream_handle(stream)), "recoil_decode")


    def decode_adaptive(self, workspace, table_index, out, err, stream=None) -> None:
        """recoil_decode_adaptive: table_index is a uint8 device tensor of N entries."""
        if table_index.numel() < self.n_symbols or table_index.element_size() != 1:
            raise ValueError("table_index must hold N bytes")
        check(_lib.recoil_decode_adaptive(self._h, C.c_void_p(workspace.data_ptr()),
                                          C.c_void_p(table_index.data_ptr()), C.c_void_p(out.data_ptr()),
                                          C.c_void_p(err.data_ptr()), _stream_handle(stream)),
              "recoil_decode_adaptive")

    def decode_count_writes(self, workspace, out, counts, err, stream=None) -> None:
        """recoil_decode_count_writes: decode and add 1 to counts[i] (int32 device tensor
        of N zeros) for every store of symbol i."""
        if counts.numel() < self.n_symbols or counts.element_size() != 4:
            raise ValueError("counts must hold N 32-bit words")
        check(_lib.recoil_decode_count_writes(self._h, C.c_void_p(workspace.data_ptr()),
                                              C.c_void_p(out.data_ptr()), C.c_void_p(counts.data_ptr()),
                                              C.c_void_p(err.data_ptr()), _stream_handle(stream)),
              "recoil_decode_count_writes")

    def layout(self) -> _lib.PlanLayout:
        """Byte offsets of the workspace sections, unit count and lanes per unit."""
        lay = _lib.PlanLayout()
        check(_lib.recoil_plan_get_layout(self._h, C.byref(lay)), "recoil_plan_get_layout")
        return lay

    def decode_table(self) -> bytes:
        """The decode table as uploaded (layout in include/recoil.h)."""
        n = C.c_size_t()
        check(_lib.recoil_plan_decode_table(self._h, None, 0, C.byref(n)), "recoil_plan_decode_table")
        buf = np.zeros(max(n.value, 1), dtype=np.uint8)
        check(_lib.recoil_plan_decode_table(self._h, _ptr(buf), n.value, C.byref(n)), "recoil_plan_decode_table")
        return buf[: n.value].tobytes()

    def device_records(self, workspace):
        """(units x 4 records, units x W lane words) read back from an uploaded workspace."""
        lay = self.layout()
        U, W = lay.unit_count, lay.lanes_per_unit
        ws = workspace[lay.units: lay.lanes + 4 * U * W].cpu().numpy()
        rec = ws[: 16 * U].view(np.uint32).reshape(U, 4)
        lanes = ws[lay.lanes - lay.units:].view(np.uint32).reshape(U, W)
        return rec.copy(), lanes.copy()

    def units(self) -> np.ndarray:
        """Per-unit records (units x 4: next, top, ghi, glo) as the kernels read them."""
        n = C.c_uint32()
        check(_lib.recoil_plan_units(self._h, None, 0, C.byref(n)), "recoil_plan_units")
        rec = np.zeros((max(n.value, 1), 4), dtype=np.uint32)
        check(_lib.recoil_plan_units(self._h, C.c_void_p(rec.ctypes.data), n.value, C.byref(n)), "recoil_plan_units")
        return rec[: n.value]


def decode_blob(blob: Blob, device="cuda"):
    """Convenience: upload, decode and return (symbols tensor, error word)."""
    import torch
    plan = Plan(blob)
    ws = plan.allocate_workspace(device)
    plan.upload(ws)
    out = plan.allocate_output(device)
    err = torch.zeros(1, dtype=torch.int32, device=device)
    plan.decode(ws, out, err)
    torch.cuda.synchronize()
    return plan.symbols_of(out), int(err.item())
