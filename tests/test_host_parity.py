"""Host-side parity: librecoil's encoder, container writer and combiner produce
exactly the oracle's bytes on seeded inputs, and its validator rejects
corrupted containers. Runs on the CPU (no kernel launches)."""

import numpy as np
import pytest

import synth


@pytest.fixture(scope="module")
def rc():
    import paper_2306_12141_amd as m
    return m


def _syms(seed, n, A, dtype=np.uint8, skew=None):
    if skew is None:
        return (synth.splitmix64(seed, 0, n) % np.uint64(A)).astype(dtype)
    return synth.draw_symbols(synth.zipf_pmf(A, skew), seed, n, dtype)


CASES = [
    # lanes, n, dtype, alphabet, N, splits, zipf
    (32, 11, np.uint8, 256, 200_000, 50, 1.1),
    (64, 12, np.uint8, 256, 200_000, 50, 0.9),
    (1, 8, np.uint8, 16, 5_000, 12, 1.0),
    (3, 10, np.uint8, 100, 20_000, 17, None),
    (17, 16, np.uint8, 256, 50_000, 9, 1.4),
    (32, 12, np.uint16, 4096, 100_000, 20, 1.2),
    (32, 16, np.uint16, 60000, 80_000, 8, None),
    (32, 11, np.uint8, 256, 10, 4, None),
    (32, 11, np.uint8, 256, 0, 1, None),
    (32, 12, np.uint8, 2, 100_000, 100, 4.0),
    (64, 4, np.uint8, 3, 30_000, 1000, 0.5),
]


@pytest.mark.parametrize("ci", range(len(CASES)))
def test_encode_byte_identical(rc, orc, ci):
    W, n, dt, A, N, M, z = CASES[ci]
    s = _syms(2000 + ci, N, A, dt, z)
    mine = rc.encode(s, lanes=W, quant_bits=n, splits=M, alphabet=A).to_bytes()
    ref = orc.encode(s, orc.params(lanes=W, quant_bits=n, symbol_bytes=dt().itemsize, alphabet=A), M).container()
    assert mine == ref


def test_c0_identical_and_combines(rc, orc):
    spec = synth.c0_spec()
    s = spec.generate()
    blob = rc.encode(s, lanes=32, quant_bits=11, splits=256)
    ref = orc.encode(s, orc.params(lanes=32, quant_bits=11), 256).container()
    assert blob.to_bytes() == ref
    for t in (255, 128, 77, 16, 3, 1, 1000):
        assert blob.combine(t).to_bytes() == orc.combine(ref, t)
    info = blob.info
    assert info.splits == 256 and info.total_bytes == len(ref)


def test_given_frequency_table(rc, orc):
    s = _syms(5, 30_000, 8)
    f = np.array([100, 200, 300, 400, 500, 300, 200, 48], dtype=np.uint32)
    assert f.sum() == 2048
    mine = rc.encode(s, lanes=32, quant_bits=11, splits=10, alphabet=8, freq=f).to_bytes()
    ref = orc.encode(s, orc.params(lanes=32, quant_bits=11, alphabet=8), 10, freq=f).container()
    assert mine == ref


def test_quantize_matches_oracle(rc, orc):
    for seed in range(20):
        A = 1 + seed * 13
        counts = (synth.splitmix64(seed, 0, A) % np.uint64(1000)).astype(np.uint64)
        counts[::3] = 0
        if counts.sum() == 0:
            continue
        for n in (8, 12, 16):
            if np.count_nonzero(counts) > (1 << n):
                continue
            assert np.array_equal(rc.quantize(counts, n), orc.quantize(counts, n))


def test_deserialize_roundtrip(rc):
    s = _syms(1, 50_000, 256, np.uint8, 1.1)
    data = rc.encode(s, lanes=32, quant_bits=11, splits=20).to_bytes()
    assert rc.Blob.from_bytes(data).to_bytes() == data


@pytest.mark.parametrize("W,N,dt", [(32, 200, np.uint8), (32, 1392, np.uint8), (64, 1392, np.uint16),
                                    (64, 5000, np.uint8), (59, 1392, np.uint16)])
def test_more_units_than_groups(rc, orc, W, N, dt):
    """A small stream asked for many splits is cut finer than its symbol groups
    (several split points in one group, some units empty). The container round-trips,
    equals the oracle's bytes, and the oracle decodes it back to the input."""
    A = 256 if dt == np.uint8 else 4096
    s = _syms(77 + W + N, N, A, dt, 1.1)
    blob = rc.encode(s, lanes=W, quant_bits=12, splits=400, alphabet=A)
    G = -(-N // W)
    assert blob.info.splits > G
    data = blob.to_bytes()
    assert data == orc.encode(s, orc.params(lanes=W, quant_bits=12, symbol_bytes=dt().itemsize, alphabet=A),
                              400).container()
    assert rc.Blob.from_bytes(data).to_bytes() == data
    assert np.array_equal(orc.Decoder(data).all(), s)
    assert np.array_equal(orc.Decoder(blob.combine(G // 2 + 1).to_bytes()).all(), s)


def test_corruption_rejected(rc):
    s = _syms(2, 50_000, 256, np.uint8, 1.1)
    data = bytearray(rc.encode(s, lanes=32, quant_bits=11, splits=20).to_bytes())
    bad = [data[:47], data[:-1], data + b"\0"]
    for off in (0, 4, 6, 7, 8, 9, 12, 24, 32, 36, 40):
        d = bytearray(data)
        d[off] ^= 0xFF
        bad.append(d)
    for d in bad:
        with pytest.raises(rc.RecoilError):
            rc.Blob.from_bytes(bytes(d))
    # Flip bits inside the metadata: must be rejected or still decode to a valid layout.
    hdr_meta = int.from_bytes(data[40:44], "little")
    tb = int.from_bytes(data[36:40], "little")
    start = 48 + tb + 4 * 32
    rejected = 0
    for k in range(0, hdr_meta, max(1, hdr_meta // 64)):
        d = bytearray(data)
        d[start + k] ^= 0x80
        try:
            rc.Blob.from_bytes(bytes(d))
        except rc.RecoilError:
            rejected += 1
    assert rejected > 0


def test_mutated_containers(rc):
    """Seeded random mutations (bit flips, overwritten runs, truncation) of several
    containers: the validator either rejects one or accepts a canonical container
    (it re-serialises to the same bytes); planning and combining it either succeed or
    return an error status."""
    rng = np.random.default_rng(31)
    blobs = [rc.encode(_syms(40 + i, N, A, dt, 1.1), lanes=W, quant_bits=n, splits=M, alphabet=A).to_bytes()
             for i, (W, n, dt, A, N, M) in enumerate([(32, 11, np.uint8, 256, 20_000, 12),
                                                       (64, 12, np.uint16, 4096, 9_000, 7),
                                                       (32, 12, np.uint8, 256, 1_392, 400)])]
    accepted = rejected = 0
    for data in blobs:
        for _ in range(150):
            d = bytearray(data)
            kind = rng.integers(4)
            if kind == 0:
                for p in rng.integers(len(d), size=rng.integers(1, 9)):
                    d[p] ^= 1 << int(rng.integers(8))
            elif kind == 1:
                d = d[:rng.integers(len(d))]
            elif kind == 2:
                p = int(rng.integers(len(d)))
                d[p:p + 16] = bytes([0xFF if rng.integers(2) else 0]) * len(d[p:p + 16])
            else:
                d[int(rng.integers(min(len(d), 256)))] = int(rng.integers(256))
            try:
                b = rc.Blob.from_bytes(bytes(d))
            except rc.RecoilError:
                rejected += 1
                continue
            accepted += 1
            assert b.to_bytes() == bytes(d)
            for step in (lambda: rc.Plan(b), lambda: b.combine(3)):
                try:
                    step()
                except rc.RecoilError:   # e.g. a header naming a stream too large to plan
                    pass
    assert accepted > 0 and rejected > 0


def test_invalid_arguments(rc):
    with pytest.raises(rc.RecoilError):
        rc.encode(np.array([300], dtype=np.uint16), lanes=32, quant_bits=11, alphabet=256)
    with pytest.raises(rc.RecoilError):
        rc.encode(np.arange(10, dtype=np.uint8), lanes=0, quant_bits=11)
    with pytest.raises(rc.RecoilError):
        rc.encode(np.arange(10, dtype=np.uint8), lanes=32, quant_bits=3)   # 10 symbols > 8 slots


def test_plan_rejects_unsupported(rc):
    s = _syms(3, 10_000, 256)
    with pytest.raises(rc.RecoilError):
        rc.Plan(rc.encode(s, lanes=16, quant_bits=11, splits=4))
    rc.Plan(rc.encode(s, lanes=32, quant_bits=13, splits=4))   # n <= 16 (Table 3), two-level table
    # Eq. 2 on the GPU multiplies f by x >> n in 24 bits, which holds only for n >= 8.
    with pytest.raises(rc.RecoilError) as e:
        rc.Plan(rc.encode(s % 64, lanes=32, quant_bits=7, splits=4, alphabet=64))
    assert e.value.status == -4
    plan = rc.Plan(rc.encode(s, lanes=32, quant_bits=11, splits=4))
    assert plan.device_bytes > 0 and plan.splits == 4


@pytest.mark.parametrize("W,N,P,dt", [(32, 100_001, 64, np.uint8), (64, 64 * 300, 300, np.uint8),
                                      (32, 50_000, 1, np.uint16), (32, 1000, 5000, np.uint8), (64, 0, 3, np.uint8)])
def test_partitioned_byte_identical(rc, orc, W, N, P, dt):
    """The conventional baseline (Sec. 2.3): librecoil's container equals the oracle's
    byte for byte, deserialises to the same bytes, plans one unit per sub-sequence
    and cannot be combined."""
    from tests import _fmt
    A = 256 if dt == np.uint8 else 4096
    s = _syms(500 + W + P, N, A, dt, skew=1.1)
    n = 12 if dt == np.uint16 else 11
    p = orc.params(lanes=W, quant_bits=n, symbol_bytes=np.dtype(dt).itemsize, alphabet=A)
    ref = orc.encode_partitioned(s, p, P)
    blob = rc.encode_partitioned(s, lanes=W, quant_bits=n, partitions=P, alphabet=A)
    assert blob.to_bytes() == ref
    assert rc.Blob.from_bytes(ref).to_bytes() == ref
    c = _fmt.parse_partitioned(ref)
    assert blob.splits == c["P"] and blob.info.metadata_bytes == c["P"] * 4 * (1 + W)
    units = rc.Plan(blob).units()
    S = c["S"]
    for q, (nxt, top, ghi, glo) in enumerate(units):
        lo, hi = q * S, min(N, (q + 1) * S)
        assert glo == lo // W and ghi == top and (hi == lo or top == (hi - 1) // W)
        assert nxt == (c["starts"][q + 1] if q + 1 < c["P"] else c["B"])
    with pytest.raises(rc.RecoilError):
        blob.combine(2)


def test_partitioned_corruption_rejected(rc, orc):
    s = _syms(61, 20_000, 256, skew=1.2)
    good = bytearray(orc.encode_partitioned(s, orc.params(lanes=32, quant_bits=11), 9))
    for off, val in [(44, 33), (32, 8), (48 + 40, 0xFF), (len(good) - 1, None)]:
        bad = bytearray(good)
        if val is None:
            bad = bad[:-1]
        elif off == 44:
            bad[44:48] = (33).to_bytes(4, "little")          # S not a multiple of W
        elif off == 32:
            bad[32:36] = (8).to_bytes(4, "little")           # P disagrees with N and S
        else:
            hdr = 48 + int.from_bytes(good[36:40], "little")   # first offset must be 0
            bad[hdr:hdr + 4] = (5).to_bytes(4, "little")
        with pytest.raises(rc.RecoilError):
            rc.Blob.from_bytes(bytes(bad))


def _adaptive_case(orc, seed, n, T, A, nbits):
    pmfs, tidx, s = synth.adaptive_stream(seed, n, T, A)
    tabs = np.stack([orc.quantize((pmf * (1 << 30)).astype(np.uint64) + 1, nbits) for pmf in pmfs])
    return tabs, tidx, s


@pytest.mark.parametrize("W,n,T,A,M", [(32, 200_001, 16, 64, 97), (64, 65_536, 4, 256, 33), (32, 5000, 1, 64, 1)])
def test_adaptive_byte_identical(rc, orc, W, n, T, A, M):
    """Adaptive coding: librecoil's container equals the oracle's, deserialises to the
    same bytes, combines like the oracle's, and plans T decode tables."""
    nbits = 9 if T == 16 else 11
    tabs, tidx, s = _adaptive_case(orc, 300 + W + T, n, T, A, nbits)
    p = orc.params(lanes=W, quant_bits=nbits, alphabet=A)
    ref = orc.encode_adaptive(s, p, tabs, tidx, M).container()
    blob = rc.encode_adaptive(s, tabs, tidx, lanes=W, quant_bits=nbits, splits=M, alphabet=A)
    assert blob.to_bytes() == ref and ref[:4] == b"RCA1"
    assert rc.Blob.from_bytes(ref).to_bytes() == ref
    assert blob.combine(7).to_bytes() == orc.combine(ref, 7)
    assert len(rc.Plan(blob).units()) == blob.splits
    with pytest.raises(rc.RecoilError):       # a table index beyond the tables
        rc.encode_adaptive(s, tabs, np.full_like(tidx, T), lanes=W, quant_bits=nbits, splits=M, alphabet=A)


def test_adaptive_plan_limits(rc, orc):
    """The GPU decodes adaptive uint8 streams whose tables fit 64 KiB of LDS."""
    tabs, tidx, s = _adaptive_case(orc, 9, 10_000, 32, 64, 10)       # 32 x 1024 x 4 B = 128 KiB
    with pytest.raises(rc.RecoilError):
        rc.Plan(rc.encode_adaptive(s, tabs, tidx, lanes=32, quant_bits=10, splits=4, alphabet=64))


@pytest.mark.parametrize("W,n,dt,A,N,M,z", [(64, 16, np.uint8, 256, 100_000, 30, 1.1),
                                            (32, 13, np.uint8, 256, 50_000, 8, None),
                                            (32, 15, np.uint16, 4096, 60_000, 9, 1.0)])
def test_wide_byte_identical_and_planned(rc, orc, W, n, dt, A, N, M, z):
    """13 <= n <= 16: containers equal the oracle's and the GPU planner accepts them."""
    s = _syms(7000 + n, N, A, dt, z)
    blob = rc.encode(s, lanes=W, quant_bits=n, splits=M, alphabet=A)
    p = orc.params(lanes=W, quant_bits=n, symbol_bytes=np.dtype(dt).itemsize, alphabet=A)
    assert blob.to_bytes() == orc.encode(s, p, M).container()
    plan = rc.Plan(blob)
    assert plan.units().shape == (blob.splits, 4)
    assert rc.Plan(blob, packed_target=0).layout().unit_count == blob.splits


def test_wide_limits(rc):
    """n > 12 decodes on the GPU only with at most 4096 symbols of f > 0 and without
    adaptive tables; batches take such streams (a table class of their own)."""
    s = (synth.splitmix64(7100, 0, 200_000) % np.uint64(60000)).astype(np.uint16)
    blob = rc.encode(s, lanes=32, quant_bits=16, splits=4, alphabet=60000)
    with pytest.raises(rc.RecoilError, match="unsupported"):
        rc.Plan(blob)
    ok = rc.encode((s % 4096).astype(np.uint16), lanes=32, quant_bits=16, splits=4, alphabet=4096)
    rc.Plan(ok)
    from paper_2306_12141_amd import batch
    assert batch.Batch([ok, rc.encode(s[:5000] % 256, lanes=32, quant_bits=11, splits=3, alphabet=4096)]).items >= 2


SPLIT_WRITER_CASES = [
    # lanes, n, dtype, alphabet, N, splits, zipf
    (32, 11, np.uint8, 256, 300_001, 64, 1.1),
    (64, 12, np.uint8, 256, 200_000, 37, 0.9),
    (1, 8, np.uint8, 16, 5_000, 12, 1.0),
    (3, 10, np.uint8, 100, 20_000, 17, None),
    (17, 16, np.uint8, 256, 50_000, 9, 1.4),
    (32, 12, np.uint16, 4096, 100_000, 20, 1.2),
    (32, 11, np.uint8, 256, 10, 4, None),
    (32, 12, np.uint8, 2, 100_000, 100, 4.0),
    (64, 4, np.uint8, 3, 30_000, 1000, 0.5),
    (32, 11, np.uint8, 256, 1 << 20, 30_000, 1.1),
]


@pytest.mark.parametrize("ci", range(len(SPLIT_WRITER_CASES)))
def test_parallel_split_writer_identical(rc, orc, ci):
    """The threaded split writer (segmented per-lane scan, then the greedy walk)
    chooses the streaming chooser's split points: containers byte-identical for
    2, 3 and 8 threads, and equal to the oracle's."""
    W, n, dt, A, N, M, z = SPLIT_WRITER_CASES[ci]
    s = _syms(9000 + ci, N, A, dt, z)
    outs = []
    try:
        for t in (1, 2, 3, 8):
            rc.set_split_writer_threads(t)
            outs.append(rc.encode(s, lanes=W, quant_bits=n, splits=M, alphabet=A).to_bytes())
    finally:
        rc.set_split_writer_threads(0)
    assert all(o == outs[0] for o in outs[1:])
    if N <= 300_001:
        p = orc.params(lanes=W, quant_bits=n, symbol_bytes=np.dtype(dt).itemsize, alphabet=A)
        assert outs[0] == orc.encode(s, p, M).container()


def test_parallel_split_writer_adaptive(rc, orc):
    pmfs, tidx, s = synth.adaptive_stream(9100, 400_000, 8, 64)
    tabs = np.stack([orc.quantize((pmf * (1 << 30)).astype(np.uint64) + 1, 10) for pmf in pmfs])
    outs = []
    try:
        for t in (1, 4):
            rc.set_split_writer_threads(t)
            outs.append(rc.encode_adaptive(s, tabs, tidx, lanes=32, quant_bits=10, splits=300, alphabet=64).to_bytes())
    finally:
        rc.set_split_writer_threads(0)
    assert outs[0] == outs[1]


def test_parallel_split_writer_sparse_events(rc):
    """Words so rare that most positions fail the 16-bit group-difference test
    (f = 2^16 - 1 for symbol 0 at n = 16): the threaded writer still chooses the
    streaming chooser's split points, including when fewer than M exist."""
    N = 1 << 21
    s = np.zeros(N, dtype=np.uint8)
    s[(synth.splitmix64(9200, 0, 64) % np.uint64(N)).astype(np.int64)] = 1
    freq = np.array([65535, 1], dtype=np.uint32)
    outs = []
    try:
        for t in (1, 2, 8):
            rc.set_split_writer_threads(t)
            for W, M in ((2, 8), (32, 64)):
                outs.append((t, W, rc.encode(s, lanes=W, quant_bits=16, splits=M, alphabet=2, freq=freq).to_bytes()))
    finally:
        rc.set_split_writer_threads(0)
    ref = {W: o for t, W, o in outs if t == 1}
    assert all(o == ref[W] for t, W, o in outs)
