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


def parse_partitioned(c: bytes) -> dict:
    """The conventional partitioned container ("RCP1"): header, table, per
    sub-sequence its first word and W final states, then the words."""
    (magic, version, lanes, n, sym_bytes, l_bits, b_bits, _r0, alphabet, N, B, P,
     table_bytes, meta_bytes, S) = HEADER.unpack_from(c, 0)
    assert magic == b"RCP1"
    off = 48 + table_bytes
    rec = np.frombuffer(c[off:off + meta_bytes], dtype="<u4").reshape(P, 1 + lanes)
    off += meta_bytes
    words = np.frombuffer(c[off:off + 2 * B], dtype="<u2")
    assert off + 2 * B == len(c)
    starts = rec[:, 0].astype(np.int64)
    ends = np.append(starts[1:], B)
    return dict(lanes=lanes, N=N, B=B, P=P, S=S, table=c[48:48 + table_bytes], starts=starts,
                final=rec[:, 1:], words=words, part_words=[words[a:b] for a, b in zip(starts, ends)])
