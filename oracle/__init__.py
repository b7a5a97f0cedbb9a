"""Python access to the Recoil CPU oracle -- TEST INFRASTRUCTURE ONLY.

Loads `liboracle.so` (plain serial C++ built from oracle.cpp) through ctypes.
Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
module; the product library never imports it.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import List, Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.cpp")


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (plain C++17, -O2, no SIMD intrinsics)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-Wall", "-shared", "-fPIC",
                               "-pthread", _SRC, "-o", tmp])
        os.replace(tmp, _SO)
    return _SO


class Params(C.Structure):
    _fields_ = [("lanes", C.c_uint32), ("quant_bits", C.c_uint32), ("symbol_bytes", C.c_uint32),
                ("alphabet", C.c_uint32), ("l_bits", C.c_uint32), ("b_bits", C.c_uint32)]


class Info(C.Structure):
    _fields_ = [("n_symbols", C.c_uint64), ("n_words", C.c_uint64), ("threads", C.c_uint32),
                ("lanes", C.c_uint32), ("quant_bits", C.c_uint32), ("symbol_bytes", C.c_uint32),
                ("alphabet", C.c_uint32), ("l_bits", C.c_uint32), ("b_bits", C.c_uint32),
                ("table_bytes", C.c_uint64), ("metadata_bytes", C.c_uint64),
                ("total_bytes", C.c_uint64)]


class Event(C.Structure):
    _fields_ = [("pos", C.c_uint64), ("lane", C.c_uint32), ("idx", C.c_int64),
                ("state", C.c_uint32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = C.CDLL(_SO)
        P = C.c_void_p
        u8p = C.POINTER(C.c_uint8)
        L.orc_quantize.argtypes = [P, C.c_uint32, C.c_uint32, P]
        L.orc_encode.argtypes = [P, C.c_uint64, C.POINTER(Params), P, C.c_uint32, C.POINTER(P)]
        L.orc_enc_free.argtypes = [P]
        L.orc_enc_free.restype = None
        L.orc_enc_container_size.argtypes = [P]
        L.orc_enc_container_size.restype = C.c_uint64
        L.orc_enc_container.argtypes = [P, P, C.c_uint64]
        L.orc_enc_threads.argtypes = [P]
        L.orc_enc_threads.restype = C.c_uint32
        L.orc_enc_num_events.argtypes = [P]
        L.orc_enc_num_events.restype = C.c_uint64
        L.orc_enc_num_candidates.argtypes = [P]
        L.orc_enc_num_candidates.restype = C.c_uint64
        L.orc_enc_events.argtypes = [P, P, C.c_uint64]
        L.orc_enc_split.argtypes = [P, C.c_uint32, P, P, P, P, P]
        L.orc_enc_candidate_at.argtypes = [P, C.c_uint64, P, P, P, P, P]
        L.orc_scan_events.argtypes = [P, C.c_uint64, C.c_uint32, C.c_uint64, P, P, P]
        L.orc_series_pack.argtypes = [P, C.c_uint64, C.c_uint32, C.c_int, P, C.c_uint64, P]
        L.orc_series_unpack.argtypes = [P, C.c_uint64, C.c_uint64, C.c_uint32, C.c_int, P, P]
        L.orc_assemble.argtypes = [C.POINTER(Params), C.c_uint64, P, P, C.c_uint64, P, C.c_uint32,
                                   P, P, P, P, C.c_uint64, P]
        L.orc_encode_adaptive.argtypes = [P, C.c_uint64, C.POINTER(Params), P, C.c_uint32, P, C.c_uint32,
                                          C.POINTER(P)]
        L.orc_set_table_index.argtypes = [P, P, C.c_uint64]
        L.orc_encode_partitioned.argtypes = [P, C.c_uint64, C.POINTER(Params), P, C.c_uint32, P, C.c_uint64, P]
        L.orc_info_of.argtypes = [P, C.c_uint64, C.POINTER(Info)]
        L.orc_combine.argtypes = [P, C.c_uint64, C.c_uint32, P, C.c_uint64, P]
        L.orc_open.argtypes = [P, C.c_uint64, C.POINTER(P)]
        L.orc_close.argtypes = [P]
        L.orc_close.restype = None
        L.orc_decode_serial.argtypes = [P, P]
        L.orc_decode_thread.argtypes = [P, C.c_uint32, C.c_int, P]
        L.orc_decode_thread_trace.argtypes = [P, C.c_uint32, C.c_int, P, P, C.c_uint64, P]
        L.orc_thread_range.argtypes = [P, C.c_uint32, C.c_int, P, P]
        L.orc_decode_all.argtypes = [P, C.c_int, C.c_uint32, P]
        del u8p
        _lib = L
    return _lib


class OracleError(RuntimeError):
    pass


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise OracleError(f"{what} failed with status {rc}")


def _ptr(a: np.ndarray) -> C.c_void_p:
    return C.c_void_p(a.ctypes.data)


def params(lanes=32, quant_bits=11, symbol_bytes=1, alphabet=256, l_bits=16, b_bits=16) -> Params:
    return Params(lanes, quant_bits, symbol_bytes, alphabet, l_bits, b_bits)


def quantize(counts: np.ndarray, n: int) -> np.ndarray:
    counts = np.ascontiguousarray(counts, dtype=np.uint64)
    f = np.zeros(len(counts), dtype=np.uint32)
    _check(lib().orc_quantize(_ptr(counts), len(counts), n, _ptr(f)), "quantize")
    return f


@dataclass
class SplitRecord:
    pos: int
    imax: int
    imin: int
    states: np.ndarray
    indices: np.ndarray


class Encoded:
    """Handle on one oracle encoding (container bytes plus the encoder's records)."""

    def __init__(self, handle: C.c_void_p, p: Params):
        self._h = handle
        self.params = p

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_enc_free(self._h)
            self._h = None

    @property
    def threads(self) -> int:
        return lib().orc_enc_threads(self._h)

    @property
    def num_candidates(self) -> int:
        return lib().orc_enc_num_candidates(self._h)

    def container(self) -> bytes:
        n = lib().orc_enc_container_size(self._h)
        if n == 0:
            raise OracleError("container does not fit the format")
        buf = np.empty(n, dtype=np.uint8)
        _check(lib().orc_enc_container(self._h, _ptr(buf), n), "container")
        return buf.tobytes()

    def events(self) -> np.ndarray:
        n = lib().orc_enc_num_events(self._h)
        arr = (Event * max(1, n))()
        _check(lib().orc_enc_events(self._h, C.cast(arr, C.c_void_p), n), "events")
        return np.array([(e.pos, e.lane, e.idx, e.state) for e in arr[:n]], dtype=np.int64).reshape(-1, 4)

    def split(self, k: int) -> SplitRecord:
        W = self.params.lanes
        pos, imax, imin = C.c_uint64(), C.c_int64(), C.c_int64()
        st = np.zeros(W, dtype=np.uint32)
        ix = np.zeros(W, dtype=np.int64)
        _check(lib().orc_enc_split(self._h, k, C.byref(pos), C.byref(imax), C.byref(imin),
                                   _ptr(st), _ptr(ix)), "split")
        return SplitRecord(pos.value, imax.value, imin.value, st, ix)

    def candidate_at(self, pos: int) -> Optional[SplitRecord]:
        W = self.params.lanes
        valid, imax, imin = C.c_int(), C.c_int64(), C.c_int64()
        st = np.zeros(W, dtype=np.uint32)
        ix = np.zeros(W, dtype=np.int64)
        _check(lib().orc_enc_candidate_at(self._h, pos, C.byref(valid), C.byref(imax), C.byref(imin),
                                          _ptr(st), _ptr(ix)), "candidate_at")
        if not valid.value:
            return None
        return SplitRecord(pos, imax.value, imin.value, st, ix)


def encode(symbols: np.ndarray, p: Params, threads: int, freq: Optional[np.ndarray] = None) -> Encoded:
    dt = np.uint8 if p.symbol_bytes == 1 else np.uint16
    symbols = np.ascontiguousarray(symbols, dtype=dt)
    h = C.c_void_p()
    fp = None
    if freq is not None:
        freq = np.ascontiguousarray(freq, dtype=np.uint32)
        fp = _ptr(freq)
    rc = lib().orc_encode(_ptr(symbols) if symbols.size else None, symbols.size, C.byref(p), fp,
                          threads, C.byref(h))
    _check(rc, "encode")
    return Encoded(h, p)


def encode_adaptive(symbols: np.ndarray, p: Params, tables: np.ndarray, tidx: np.ndarray,
                    threads: int) -> Encoded:
    """Adaptive coding (Sec. 3.1): tables is (T, A) uint32, symbol i uses table tidx[i]."""
    dt = np.uint8 if p.symbol_bytes == 1 else np.uint16
    symbols = np.ascontiguousarray(symbols, dtype=dt)
    tables = np.ascontiguousarray(tables, dtype=np.uint32)
    tidx = np.ascontiguousarray(tidx, dtype=np.uint8)
    assert tables.ndim == 2 and tables.shape[1] == p.alphabet and len(tidx) == len(symbols)
    h = C.c_void_p()
    _check(lib().orc_encode_adaptive(_ptr(symbols) if symbols.size else None, symbols.size, C.byref(p),
                                     _ptr(tables), tables.shape[0], _ptr(tidx) if tidx.size else None, threads,
                                     C.byref(h)), "encode_adaptive")
    return Encoded(h, p)


def encode_partitioned(symbols: np.ndarray, p: Params, partitions: int,
                       freq: Optional[np.ndarray] = None) -> bytes:
    """Conventional partitioned container (Sec. 2.3): independent sub-sequences."""
    dt = np.uint8 if p.symbol_bytes == 1 else np.uint16
    symbols = np.ascontiguousarray(symbols, dtype=dt)
    fp = None
    if freq is not None:
        freq = np.ascontiguousarray(freq, dtype=np.uint32)
        fp = _ptr(freq)
    n = C.c_uint64()
    sp = _ptr(symbols) if symbols.size else None
    _check(lib().orc_encode_partitioned(sp, symbols.size, C.byref(p), fp, partitions, None, 0, C.byref(n)),
           "encode_partitioned")
    buf = np.empty(n.value, dtype=np.uint8)
    _check(lib().orc_encode_partitioned(sp, symbols.size, C.byref(p), fp, partitions, _ptr(buf), n.value,
                                        C.byref(n)), "encode_partitioned")
    return buf.tobytes()


def scan_events(events: List[Tuple[int, int, int, int]], lanes: int, split_event: int):
    """events: (pos, lane, idx, state) in word order. Returns (states, indices, valid)."""
    arr = (Event * len(events))()
    for k, (pos, lane, idx, state) in enumerate(events):
        arr[k] = Event(pos, lane, idx, state)
    st = np.zeros(lanes, dtype=np.uint32)
    ix = np.zeros(lanes, dtype=np.int64)
    valid = C.c_int()
    _check(lib().orc_scan_events(C.cast(arr, C.c_void_p), len(events), lanes, split_event,
                                 _ptr(st), _ptr(ix), C.byref(valid)), "scan_events")
    return st, ix, bool(valid.value)


def series_pack(values, width_field: int, signed: bool) -> Tuple[bytes, int]:
    v = np.ascontiguousarray(values, dtype=np.int64)
    buf = np.zeros(16 + len(v) * 5, dtype=np.uint8)
    nbits = C.c_uint64()
    _check(lib().orc_series_pack(_ptr(v), len(v), width_field, int(signed), _ptr(buf), len(buf),
                                 C.byref(nbits)), "series_pack")
    return buf[: (nbits.value + 7) // 8].tobytes(), nbits.value


def series_unpack(data: bytes, count: int, width_field: int, signed: bool) -> Tuple[np.ndarray, int]:
    src = np.frombuffer(data, dtype=np.uint8).copy()
    out = np.zeros(count, dtype=np.int64)
    nbits = C.c_uint64()
    _check(lib().orc_series_unpack(_ptr(src), len(src), count, width_field, int(signed), _ptr(out),
                                   C.byref(nbits)), "series_unpack")
    return out, nbits.value


def assemble(p: Params, n_symbols: int, freq, words, final_states, split_pos, split_states,
             split_indices) -> bytes:
    freq = np.ascontiguousarray(freq, dtype=np.uint32)
    words = np.ascontiguousarray(words, dtype=np.uint16)
    fin = np.ascontiguousarray(final_states, dtype=np.uint32)
    sp = np.ascontiguousarray(split_pos, dtype=np.uint64)
    ss = np.ascontiguousarray(split_states, dtype=np.uint32).reshape(-1)
    si = np.ascontiguousarray(split_indices, dtype=np.int64).reshape(-1)
    cap = 1 << 20
    buf = np.zeros(cap, dtype=np.uint8)
    written = C.c_uint64()
    _check(lib().orc_assemble(C.byref(p), n_symbols, _ptr(freq), _ptr(words) if words.size else None,
                              words.size, _ptr(fin), len(sp) + 1, _ptr(sp) if sp.size else None,
                              _ptr(ss) if ss.size else None, _ptr(si) if si.size else None,
                              _ptr(buf), cap, C.byref(written)), "assemble")
    return buf[: written.value].tobytes()


def info(container: bytes) -> Info:
    c = np.frombuffer(container, dtype=np.uint8)
    out = Info()
    _check(lib().orc_info_of(_ptr(c), len(c), C.byref(out)), "info")
    return out


def combine(container: bytes, target_threads: int) -> bytes:
    c = np.frombuffer(container, dtype=np.uint8)
    buf = np.empty(len(c) + 64, dtype=np.uint8)
    written = C.c_uint64()
    _check(lib().orc_combine(_ptr(c), len(c), target_threads, _ptr(buf), len(buf), C.byref(written)),
           "combine")
    return buf[: written.value].tobytes()


class Decoder:
    """Parsed container; serial and per-thread decoding."""

    def __init__(self, container: bytes):
        self._buf = np.frombuffer(container, dtype=np.uint8).copy()
        self._h = C.c_void_p()
        _check(lib().orc_open(_ptr(self._buf), len(self._buf), C.byref(self._h)), "open")
        self.info = info(container)
        self.dtype = np.uint8 if self.info.symbol_bytes == 1 else np.uint16

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_close(self._h)
            self._h = None

    @property
    def threads(self) -> int:
        return self.info.threads

    def set_table_index(self, tidx: np.ndarray) -> None:
        """Adaptive containers: the per-symbol table index decoding needs."""
        self._tidx = np.ascontiguousarray(tidx, dtype=np.uint8)
        _check(lib().orc_set_table_index(self._h, _ptr(self._tidx) if self._tidx.size else None, self._tidx.size),
               "set_table_index")

    def _out(self, fill: Optional[int]) -> np.ndarray:
        n = int(self.info.n_symbols)
        if fill is None:
            return np.zeros(max(n, 1), dtype=self.dtype)
        return np.full(max(n, 1), fill, dtype=self.dtype)

    def serial(self) -> np.ndarray:
        out = self._out(None)
        _check(lib().orc_decode_serial(self._h, _ptr(out)), "decode_serial")
        return out[: self.info.n_symbols]

    def thread_range(self, t: int, aligned: bool = False) -> Tuple[int, int]:
        lo, hi = C.c_uint64(), C.c_uint64()
        _check(lib().orc_thread_range(self._h, t, int(aligned), C.byref(lo), C.byref(hi)), "range")
        return lo.value, hi.value

    def thread(self, t: int, aligned: bool = False, out: Optional[np.ndarray] = None,
               fill: Optional[int] = None) -> np.ndarray:
        if out is None:
            out = self._out(fill)
        _check(lib().orc_decode_thread(self._h, t, int(aligned), _ptr(out)), "decode_thread")
        return out

    def thread_trace(self, t: int, aligned: bool = False) -> Tuple[np.ndarray, np.ndarray]:
        """Decode thread t; returns (buffer, indices of every symbol decoded in order)."""
        out = self._out(None)
        cap = int(self.info.n_symbols) + 64
        idx = np.zeros(cap, dtype=np.int64)
        cnt = C.c_uint64()
        _check(lib().orc_decode_thread_trace(self._h, t, int(aligned), _ptr(out), _ptr(idx), cap,
                                             C.byref(cnt)), "decode_thread_trace")
        return out, idx[: cnt.value]

    def all(self, aligned: bool = False, workers: int = 1, fill: Optional[int] = None) -> np.ndarray:
        out = self._out(fill)
        _check(lib().orc_decode_all(self._h, int(aligned), workers, _ptr(out)), "decode_all")
        return out[: self.info.n_symbols]
