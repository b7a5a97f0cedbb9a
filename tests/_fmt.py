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


class BitReader:
    """MSB-first reader of a packed section."""

    def __init__(self, data: bytes):
        self.s = bits(data)
        self.pos = 0

    def get(self, w: int) -> int:
        v = int(self.s[self.pos:self.pos + w], 2)
        self.pos += w
        return v

    def series(self, count: int, field: int, signed: bool) -> list:
        w = self.get(field) + 1
        out = []
        for _ in range(count):
            neg = self.get(1) if signed else 0
            m = self.get(w)
            out.append(-m if neg else m)
        return out


def unit_records(c: bytes, target: int = 0):
    """Per-unit records (next, top, ghi, glo) and lane words that a decoder of the
    container combined to `target` units starts from, read straight from the
    packed metadata section: offset and group series, then per split point W
    16-bit states and a group-difference series (Sec. 4.3 layout in
    include/recoil.h). Every ceil(M / target)-th split point is kept (0: all)."""
    h = parse(c)
    W, M, B, N = h["lanes"], h["M"], h["B"], h["N"]
    G = -(-N // W)
    r = BitReader(h["meta"])
    o = r.series(M - 1, 5, True) if M > 1 else []
    x = r.series(M - 1, 5, True) if M > 1 else []
    states, diffs = [], []
    for _ in range(M - 1):
        states.append([r.get(16) for _ in range(W)])
        diffs.append(r.series(W, 4, False))
    eb, eg = -(-B // M), -(-G // M)
    step = -(-M // (M if target == 0 else min(target, M)))
    units = (M - 1) // step + 1
    rec = np.zeros((units, 4), dtype=np.uint32)
    lanes = np.zeros((units, W), dtype=np.uint32)
    prev_sync = None
    for u in range(units):
        glo = 0 if u == 0 else prev_sync + 1
        if u + 1 == units:
            rec[u] = (B, max(G - 1, 0), max(G - 1, 0), glo)
            lanes[u] = h["final"]
            continue
        k = (u + 1) * step - 1
        top = (k + 1) * eg + x[k] - 1
        ghi = top - max(diffs[k])
        rec[u] = ((k + 1) * eb + o[k], top, ghi, glo)
        lanes[u] = [s | (d << 16) for s, d in zip(states[k], diffs[k])]
        prev_sync = ghi
    return rec, lanes
