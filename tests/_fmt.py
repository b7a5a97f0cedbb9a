"""Container layout reader used by the tests (the byte layout is specified in include/recoil.h)."""

import struct

import numpy as np

HEADER = struct.Struct("<4sHBBBBBBIQQIIII")
assert HEADER.size == 48


def parse(c: bytes) -> dict:
    (magic, version, lanes, n, sym_bytes, l_bits, b_bits, _r0, alphabet, N, B, M,
     table_bytes, meta_bytes, _r1) = HEADER.unpack_from(c, 0)
    off = 48
    table = c[off:off + table_bytes]
    off += table_bytes
    final = np.frombuffer(c[off:off + 4 * lanes], dtype="<u4")
    off += 4 * lanes
    meta = c[off:off + meta_bytes]
    off += meta_bytes
    words = np.frombuffer(c[off:off + 2 * B], dtype="<u2")
    off += 2 * B
    assert off == len(c)
    return dict(magic=magic, version=version, lanes=lanes, quant_bits=n, symbol_bytes=sym_bytes,
                l_bits=l_bits, b_bits=b_bits, alphabet=alphabet, N=N, B=B, M=M, table=table,
                final=final, meta=meta, words=words)


def bits(data: bytes, nbits: int = None) -> str:
    s = "".join(f"{b:08b}" for b in data)
    return s if nbits is None else s[:nbits]
