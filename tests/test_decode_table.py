"""The GPU decode tables (Eq. 2: slot -> symbol s with F(s) <= slot < F(s) + f(s),
and f(s), slot - F(s)), checked slot by slot against a cumulative search over the
container's own frequency table. Covers the one-level tables of n <= 12 (uint8
and uint16 entries, adaptive tables laid end to end) and the two-level tables of
13 <= n <= 16 (16-slot buckets, then one entry per symbol with f > 0; the lookup
below follows the layout documented in include/recoil.h). Runs on the CPU.
"""

import numpy as np
import pytest

import synth
from tests._fmt import BitReader, parse


@pytest.fixture(scope="module")
def rc():
    import paper_2306_12141_amd as m
    return m


def _freqs(container: bytes, tables: int = 1):
    h = parse(container)
    r = BitReader(h["table"])
    return [np.array(r.series(h["alphabet"], 5, False), dtype=np.int64) for _ in range(tables)], h


def _truth(freq):
    """(symbol, f, slot - F) of every slot by searching the cumulative frequencies."""
    cum = np.concatenate([[0], np.cumsum(freq)])
    slots = np.arange(int(cum[-1]))
    sym = np.searchsorted(cum, slots, side="right") - 1
    return sym, freq[sym], slots - cum[sym]


def _wide_lookup(table: bytes, n: int):
    nb = 1 << (n - 4)
    w = np.frombuffer(table, dtype="<u4")
    buckets, ranks = w[:nb].astype(np.int64), w[nb:]
    slots = np.arange(1 << n)
    c = buckets[slots >> 4]
    p = slots & 15
    low = c & ((1 << p) - 1)
    pop = np.array([bin(int(v)).count("1") for v in low])
    r = (c >> 16) + pop
    f = ranks[2 * r].astype(np.int64)
    y = ranks[2 * r + 1].astype(np.int64)
    return y & 0xFFFF, f, slots - (y >> 16)


def _syms(seed, n, A, dtype, skew):
    if skew is None:
        return (synth.splitmix64(seed, 0, n) % np.uint64(A)).astype(dtype)
    return synth.draw_symbols(synth.zipf_pmf(A, skew), seed, n, dtype)


@pytest.mark.parametrize("n,dt,A,skew", [(13, np.uint8, 256, 1.1), (16, np.uint8, 256, 1.1), (16, np.uint8, 256, None),
                                         (14, np.uint8, 3, 2.0), (15, np.uint16, 4096, 1.0), (16, np.uint16, 4096, None),
                                         (13, np.uint16, 4096, None), (16, np.uint16, 60, 0.5)])
def test_wide_table_every_slot(rc, n, dt, A, skew):
    s = _syms(8000 + n, 100_000, A, dt, skew)
    blob = rc.encode(s, lanes=32, quant_bits=n, splits=5, alphabet=A)
    (freq,), _ = _freqs(blob.to_bytes())
    assert freq.sum() == 1 << n
    table = rc.Plan(blob).decode_table()
    present = int((freq > 0).sum())
    assert len(table) == -(-(4 * (1 << (n - 4)) + 8 * present) // 16) * 16
    got = _wide_lookup(table, n)
    for g, t, what in zip(got, _truth(freq), ("symbol", "f", "slot - F")):
        assert np.array_equal(g, t), what


@pytest.mark.parametrize("n,dt,A", [(11, np.uint8, 256), (12, np.uint8, 200), (8, np.uint8, 5),
                                    (12, np.uint16, 4096), (10, np.uint16, 1000)])
def test_plain_table_every_slot(rc, n, dt, A):
    s = _syms(8100 + n, 100_000, A, dt, 1.0)
    blob = rc.encode(s, lanes=64, quant_bits=n, splits=5, alphabet=A)
    (freq,), _ = _freqs(blob.to_bytes())
    table = rc.Plan(blob).decode_table()
    if dt == np.uint8:
        e = np.frombuffer(table, dtype="<u4").astype(np.int64)
        got = (e & 0xFF, (e >> 8) & 0xFFF, e >> 20)
    else:
        e = np.frombuffer(table, dtype="<u4").astype(np.int64).reshape(-1, 2)
        got = (e[:, 1], e[:, 0] & 0xFFFF, e[:, 0] >> 16)
    for g, t, what in zip(got, _truth(freq), ("symbol", "f", "slot - F")):
        assert np.array_equal(g, t), what


def test_adaptive_tables_every_slot(rc, orc):
    T, A, nbits = 8, 64, 10
    pmfs, tidx, s = synth.adaptive_stream(8200, 50_000, T, A)
    tabs = np.stack([orc.quantize((pmf * (1 << 30)).astype(np.uint64) + 1, nbits) for pmf in pmfs])
    blob = rc.encode_adaptive(s, tabs, tidx, lanes=32, quant_bits=nbits, splits=4, alphabet=A)
    e = np.frombuffer(rc.Plan(blob).decode_table(), dtype="<u4").astype(np.int64).reshape(T, 1 << nbits)
    for t in range(T):
        sym, f, off = _truth(tabs[t].astype(np.int64))
        assert np.array_equal(e[t] & 0xFF, sym) and np.array_equal((e[t] >> 8) & 0xFFF, f)
        assert np.array_equal(e[t] >> 20, off)
