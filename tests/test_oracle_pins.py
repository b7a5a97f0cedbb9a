"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: the paper's
worked example (Sec. 4.1 figure walk-through, the two metadata tables, the
displayed bit series of Sec. 4.3), closed forms of rANS on uniform tables,
Lemma 3.1, information-theoretic size bounds, and exhaustive enumeration on
tiny parameters.
"""

import itertools
import json
import math
import os

import numpy as np
import pytest

import synth
from tests import _fmt

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_recoil_example.json")


def _rng_symbols(seed, n, A, dtype=np.uint8):
    return (synth.splitmix64(seed, 0, n) % np.uint64(A)).astype(dtype)


# ---------------------------------------------------------------------------
# Closed forms (Eq. 1 and Eq. 3 with f = 1 and n = 8: each symbol appends one byte)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("lanes", [1, 2, 3, 32])
def test_uniform_closed_form_words(orc, lanes):
    """With 256 symbols of f = 1 at n = 8 every encode step is x -> 256 x + s.

    Starting from L = 2^16 a lane emits its first symbol alone before its
    second symbol, and then the two bytes s_{2m-1}, s_{2m} before symbol 2m+1;
    within a group, lanes emit in increasing order (Sec. 2.2).
    """
    N = 40 * lanes + 3
    s = _rng_symbols(11 + lanes, N, 256)
    p = orc.params(lanes=lanes, quant_bits=8, alphabet=256)
    enc = orc.encode(s, p, 1, freq=np.ones(256, dtype=np.uint32))
    words = _fmt.parse(enc.container())["words"]
    expect = []
    groups = -(-N // lanes)
    for m in range(1, groups, 2):                       # emitting groups 1, 3, 5, ...
        for j in range(lanes):
            if m * lanes + j >= N:
                continue
            local = s[j::lanes]
            if m == 1:
                expect.append(int(local[0]))
            else:
                expect.append((int(local[m - 2]) << 8) | int(local[m - 1]))
    assert words.tolist() == expect
    dec = orc.Decoder(enc.container())
    assert np.array_equal(dec.serial(), s)


def test_uniform_size_is_exact(orc):
    """f = 2^(n-8) for all 256 symbols: every symbol costs 8 bits.

    At n = 8 each step is x -> 256 x + s and at n > 8 it is
    256 x - 255 (x mod f) + s f; both are 256 x to within a factor
    1 + 2^n / x, so the code length is 8 N up to a small fraction of a bit.
    """
    for n in (8, 10, 12):
        N, W = 4096, 4
        s = _rng_symbols(n, N, 256)
        f = np.full(256, 1 << (n - 8), dtype=np.uint32)
        enc = orc.encode(s, orc.params(lanes=W, quant_bits=n), 1, freq=f)
        c = _fmt.parse(enc.container())
        # 16 B + sum_j log2(final_j) - 16 W is the code length (every lane starts at 2^16).
        total = 16 * c["B"] + sum(math.log2(int(x)) for x in c["final"]) - 16 * W
        # Per step |log2(x'/x) - 8| <= log2(e) * 2^(n-8) / x with x >= L = 2^16.
        assert abs(total - 8 * N) <= N * 1.4427 * 2.0 ** (n - 8) / 2.0 ** 16


# ---------------------------------------------------------------------------
# Quantisation
# ---------------------------------------------------------------------------

def test_quantize_properties(orc):
    counts = np.array([0, 5, 1, 0, 100, 7, 3, 0, 1], dtype=np.uint64)
    for n in (4, 8, 11, 16):
        f = orc.quantize(counts, n)
        assert int(f.sum()) == 1 << n
        assert all((f[i] > 0) == (counts[i] > 0) for i in range(len(counts)))
    # Proportional counts quantise exactly.
    f = orc.quantize(np.array([1, 1, 2, 4], dtype=np.uint64), 3)
    assert f.tolist() == [1, 1, 2, 4]
    with pytest.raises(orc.OracleError):
        orc.quantize(np.ones(9, dtype=np.uint64), 3)       # 9 symbols > 2^3 slots


@pytest.mark.parametrize("counts,n,expect", [
    # Shortfall, equal remainders: 3 x floor(8/3) = 6 < 8; the two missing units go to
    # the smaller symbols first (a larger-symbol-first rule would give [2, 3, 3]).
    ([1, 1, 1], 3, [3, 3, 2]),
    # Shortfall ordered by remainder, not by count: 16 c / 10 = 8 r0, 4 r8, 3 r2; the
    # one missing unit goes to the largest remainder, symbol 1 (by count it would be [9, 4, 3]).
    ([5, 3, 2], 4, [8, 5, 3]),
    # Excess, tie on the largest f: 8 c / 23 = 3, 3 and three rare symbols raised to 1 sum
    # to 9; the one unit comes off the smaller symbol (larger-symbol-first: [3, 2, 1, 1, 1]).
    ([10, 10, 1, 1, 1], 3, [2, 3, 1, 1, 1]),
    # Excess taken from the largest f, not the smallest f > 1: 8 c / 33 = 4, 2, 0 -> 1 x 3
    # sums to 9 (smallest-first would give [4, 1, 1, 1, 1]).
    ([20, 10, 1, 1, 1], 3, [3, 2, 1, 1, 1]),
    # Excess of two over a tie: 8 c / 24 = 3, 3, then 1 x 4 = 10; the first unit comes off
    # symbol 0, which leaves symbol 1 the unique largest for the second.
    ([10, 10, 1, 1, 1, 1], 3, [2, 2, 1, 1, 1, 1]),
])
def test_quantize_tie_breaks(orc, counts, n, expect):
    """The quantisation rule, worked by hand: f = max(1, floor(c 2^n / N)); a shortfall
    is handed out by largest remainder c 2^n mod N (ties: smaller symbol); an excess is
    removed one unit at a time from the largest f > 1 (ties: smaller symbol)."""
    f = orc.quantize(np.array(counts, dtype=np.uint64), n)
    assert f.tolist() == expect


# ---------------------------------------------------------------------------
# The paper's worked example (Sec. 4.1, Tables 1-2, Sec. 4.3)
# ---------------------------------------------------------------------------

def _golden():
    with open(GOLDEN) as fh:
        return json.load(fh)


def test_backward_scan_example(orc):
    g = _golden()
    W = g["lanes"]
    events = [(e["offset"] - 1, e["encoder"] - 1, e["symbol"] - 1, 1000 + e["symbol"])
              for e in g["events_in_word_order"]]
    split = g["split_offset"] - 1
    states, idx, valid = orc.scan_events(events, W, split)
    assert valid
    assert (idx + 1).tolist() == g["expected_recorded_symbol_per_encoder"]
    assert (states - 1000).tolist() == g["expected_recorded_symbol_per_encoder"]
    groups = -(-(idx + 1) // W)                          # 1-based group id = ceil(i / W)
    assert groups.tolist() == g["expected_group_ids"]
    assert int(groups.max()) == g["expected_anchor"]
    assert (groups - groups.max()).tolist() == g["expected_group_differences"]
    lo, hi = g["synchronisation_section"]
    assert int(idx.min()) + 1 == lo and int(idx.max()) + 1 == hi


def test_metadata_tables_and_series_bits(orc):
    """Tables 1 and 2 and the displayed series, through the container writer.

    With B = 10 words, G = 9 groups (N = 36) and M = 2 threads, the expected
    offset ceil(B/M) = 5 and the expected max group id ceil(G/M) = 5 match the
    'Expected' column of Table 1.
    """
    g = _golden()
    W = g["lanes"]
    p = orc.params(lanes=W, quant_bits=2, alphabet=4, l_bits=16, b_bits=16)
    idx = np.array(g["expected_recorded_symbol_per_encoder"]) - 1
    states = np.array([0x1111, 0x2222, 0x3333, 0x4444], dtype=np.uint32)
    c = orc.assemble(p, 36, [1, 1, 1, 1], np.arange(10), [1 << 16] * W,
                     [g["split_offset"] - 1], states[None, :], idx[None, :])
    meta = _fmt.parse(c)["meta"]
    t1 = g["split_point_metadata"]
    d_off = t1["bitstream_offset"]["difference"]
    d_grp = t1["max_symbol_group_id"]["difference"]
    # Signed series: 5-bit (width-1) field, then sign + magnitude per value.
    expect = "00000" + ("1" if d_off < 0 else "0") + format(abs(d_off), "b")
    expect += "00000" + ("1" if d_grp < 0 else "0") + format(abs(d_grp), "b")
    expect += "".join(format(int(x), "016b") for x in states)
    expect += g["group_difference_series_bits"]
    assert _fmt.bits(meta, len(expect)) == expect
    assert len(meta) == -(-len(expect) // 8)


def test_series_example_and_roundtrip(orc):
    g = _golden()
    data, nbits = orc.series_pack([1, 0, 1, 0], 4, signed=False)
    assert nbits == 8 and _fmt.bits(data) == g["group_difference_series_bits"]
    data, nbits = orc.series_pack([0, 0, 0], 4, signed=False)
    assert _fmt.bits(data, nbits) == "0000000"           # zero still takes one bit
    vals = [5, -3, 0, 1 << 20, -(1 << 31)]
    data, nbits = orc.series_pack(vals, 5, signed=True)
    assert nbits == 5 + len(vals) * (1 + 32)
    back, used = orc.series_unpack(data, len(vals), 5, signed=True)
    assert back.tolist() == vals and used == nbits
    with pytest.raises(orc.OracleError):
        orc.series_pack([1 << 16], 4, signed=False)      # 17 bits do not fit a 4-bit width field


def _find_figure6_sequence(orc):
    """A seeded sequence whose encoding holds the Figure 6 event pattern (W = 4)."""
    p = orc.params(lanes=4, quant_bits=3, alphabet=3, l_bits=4, b_bits=4)
    f = np.array([1, 2, 5], dtype=np.uint32)
    want = (np.array(_golden()["expected_recorded_symbol_per_encoder"]) - 1).tolist()
    for seed in range(5000):
        s = _rng_symbols(seed, 40, 3)
        enc = orc.encode(s, p, 1, freq=f)
        ev = enc.events()
        for k in np.nonzero(ev[:, 2] == max(want))[0]:
            cand = enc.candidate_at(int(k))
            if cand is not None and cand.indices.tolist() == want and 11 - 1 in ev[:k, 2]:
                return p, f, s, enc, cand
    raise AssertionError("no sequence with the example's pattern")


def test_synchronisation_phase_example(orc):
    """Decoding from the example split: the sync phase yields s16, s14, s12, s11, s10, s9
    and skips s15 and s13 (1-based), then continues normally."""
    g = _golden()
    p, f, s, enc, cand = _find_figure6_sequence(orc)
    c = orc.assemble(p, len(s), f, _fmt.parse(enc.container())["words"], _fmt.parse(enc.container())["final"],
                     [cand.pos], cand.states[None, :], cand.indices[None, :])
    dec = orc.Decoder(c)
    assert dec.threads == 2
    _, trace = dec.thread_trace(1)
    lo, hi = g["synchronisation_section"]
    in_sync = [int(i) + 1 for i in trace if lo <= int(i) + 1 <= hi]
    assert sorted(in_sync, reverse=True) == g["sync_phase_decoded"]
    assert not set(g["sync_phase_skipped"]) & set(in_sync)
    # After the section the thread decodes every index down to 1 exactly once.
    below = [int(i) + 1 for i in trace if int(i) + 1 < lo]
    assert sorted(below) == list(range(1, lo))
    assert np.array_equal(dec.all(), s)
    assert np.array_equal(dec.all(aligned=True), s)


# ---------------------------------------------------------------------------
# Lemma 3.1, sizes, heuristic and combining on a realistic stream
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def c0(orc):
    spec = synth.c0_spec()
    s = spec.generate()
    p = orc.params(lanes=spec.lanes, quant_bits=spec.quant_bits)
    enc = orc.encode(s, p, spec.splits)
    return spec, s, p, enc, enc.container()


def test_lemma_3_1_states_bounded(orc, c0):
    spec, s, p, enc, c = c0
    ev = enc.events()
    assert (ev[:, 3] >= 1).all() and (ev[:, 3] < (1 << 16)).all()
    for k in range(1, enc.threads):
        sp = enc.split(k)
        assert (sp.states >= 1).all() and (sp.states < (1 << 16)).all()


def test_size_against_entropy(orc, c0):
    """16 B + sum log2(final) - 16 W equals the ideal code length up to rounding."""
    spec, s, p, enc, c = c0
    hdr = _fmt.parse(c)
    f = orc.quantize(np.bincount(s, minlength=256).astype(np.uint64), spec.quant_bits)
    ideal = float(-np.log2(f[s].astype(np.float64) / (1 << spec.quant_bits)).sum())
    measured = 16 * hdr["B"] + float(np.log2(hdr["final"].astype(np.float64)).sum()) - 16 * spec.lanes
    assert abs(measured - ideal) / ideal < 1e-3
    emp = np.bincount(s, minlength=256) / len(s)
    h = -(emp[emp > 0] * np.log2(emp[emp > 0])).sum()
    assert 16 * hdr["B"] / len(s) < h * 1.01 + 0.01


# Def. 4.1 on closed-form streams, worked by hand. With f = 1 at n = 8 lane j
# emits one word before each of its local symbols 1, 3, 5, ... (0-based), i.e.
# in the odd groups m, lanes in increasing order, so word w belongs to group
# m = 2 floor(w / W) + 1 and lane j = w mod W, and records the lane's previous
# symbol, index (m - 1) W + j (the event attribution of the worked example).
# Word w is usable once every lane has an event. At word w: Imax = (m - 1) W + j;
# Imin = (m - 1) W if j = W - 1, else (m - 3) W + j + 1 (lane j + 1's event of
# the previous odd group). For W = 2: Imax = 4 floor(w/2) + j, t_s = Imax - Imin + 1
# = 2 (j = 1) or 4 (j = 0), and for the first split t = Imax + 1.
#   N = 40, two units, T = 20:  j = 1: H = |4q + 2 - 20| + |4q - 20| -> 2 at q = 5;
#                                j = 0: H = |4q - 19| + |4q - 23|     -> >= 4.
#   so the split is word 11 (Imax 21, Imin 20).
#   N = 60, three units: first T = 20 -> word 11 again; then T = ceil(38 / 2) = 19 and
#   t = Imax - 21: j = 1: H = |4q - 39| + |4q - 41| -> 2 at q = 10 (word 21, Imax 41);
#   j = 0: H = |4q - 40| + |4q - 44| -> >= 4.
# For W = 1 every event is its own lane's only one: word w has Imax = Imin = 2w,
# t_s = 1, t = 2w + 1; N = 40, T = 20: H = |2w - 19| + |2w - 20| -> 1 at w = 10.
@pytest.mark.parametrize("lanes,N,units,expect", [
    (2, 40, 2, [(11, 21, 20)]),
    (2, 60, 3, [(11, 21, 20), (21, 41, 40)]),
    (1, 40, 2, [(10, 20, 20)]),
])
def test_heuristic_hand_worked(orc, lanes, N, units, expect):
    s = _rng_symbols(21 + N, N, 256)
    p = orc.params(lanes=lanes, quant_bits=8, alphabet=256)
    enc = orc.encode(s, p, units, freq=np.ones(256, dtype=np.uint32))
    assert enc.threads == units
    got = [(enc.split(k).pos, enc.split(k).imax, enc.split(k).imin) for k in range(1, units)]
    assert got == expect
    assert np.array_equal(orc.Decoder(enc.container()).all(), s)


def test_heuristic_recomputes_target(orc):
    """Def. 4.1 with T taken from the symbols that remain (reading 7), worked by hand
    on the W = 1 closed-form stream, where word w has Imax = Imin = 2w and t_s = 1.

    N = 13, three units. Split 1: T = ceil(13 / 3) = 5, t = 2w + 1,
    H = |2w - 4| + |2w - 5| is 1 at w = 2 (Imax 4). Split 2: T = ceil((13 - 5) / 2) = 4,
    t = 2w - 4, H = |2w - 8| + |2w - 9| is 1 at w = 4 (Imax 8): units of 5, 4 and 4
    symbols. A fixed T = 5 would give H = |2w - 9| + |2w - 10|, smallest at w = 5
    (Imax 10), and units of 5, 6 and 2 symbols.
    """
    N = 13
    s = _rng_symbols(1313, N, 256)
    p = orc.params(lanes=1, quant_bits=8, alphabet=256)
    enc = orc.encode(s, p, 3, freq=np.ones(256, dtype=np.uint32))
    assert enc.threads == 3
    got = [(enc.split(k).pos, enc.split(k).imax) for k in (1, 2)]
    assert got == [(2, 4), (4, 8)]
    dec = orc.Decoder(enc.container())
    assert [dec.thread_range(t) for t in (1, 2, 3)] == [(0, 4), (4, 8), (8, 13)]
    assert np.array_equal(dec.all(), s)


def test_heuristic_properties(orc, c0):
    spec, s, p, enc, c = c0
    dec = orc.Decoder(c)
    assert dec.threads == spec.splits
    ranges = [dec.thread_range(t) for t in range(1, dec.threads + 1)]
    assert ranges[0][0] == 0 and ranges[-1][1] == len(s)
    assert all(ranges[k][1] == ranges[k + 1][0] for k in range(len(ranges) - 1))
    sizes = np.array([hi - lo for lo, hi in ranges])
    assert sizes.max() / sizes.mean() < 1.10


def test_metadata_bytes_per_split_band(orc, c0):
    """Paper Tables 5/6: Recoil metadata is about 75-88 bytes per split at W = 32."""
    spec, s, p, enc, c = c0
    per_split = orc.info(c).metadata_bytes / (spec.splits - 1)
    assert 60 <= per_split <= 100


def test_round_trip_and_every_thread(orc, c0):
    spec, s, p, enc, c = c0
    dec = orc.Decoder(c)
    assert np.array_equal(dec.serial(), s)
    assert np.array_equal(dec.all(fill=0xAB), s)
    assert np.array_equal(dec.all(aligned=True, fill=0xCD), s)
    assert np.array_equal(dec.all(workers=4), s)


@pytest.mark.parametrize("target", [128, 100, 64, 16, 3, 1])
def test_combine(orc, c0, target):
    spec, s, p, enc, c = c0
    cc = orc.combine(c, target)
    d0, d1 = orc.Decoder(c), orc.Decoder(cc)
    step = -(-spec.splits // target)
    assert d1.threads == -(-spec.splits // step)
    b0 = {d0.thread_range(t)[1] for t in range(1, d0.threads + 1)}
    b1 = {d1.thread_range(t)[1] for t in range(1, d1.threads + 1)}
    assert b1 <= b0                                      # kept split points are original ones
    assert np.array_equal(d1.all(fill=0x11), s)
    assert np.array_equal(d1.all(aligned=True), s)
    info0, info1 = orc.info(c), orc.info(cc)
    assert info1.n_words == info0.n_words                # the bitstream is untouched
    assert _fmt.parse(cc)["words"].tobytes() == _fmt.parse(c)["words"].tobytes()


@pytest.mark.parametrize("target,step,kept", [
    (100, 3, list(range(3, 256, 3))),          # 85 split points 3, 6, ..., 255: 86 units
    (7, 37, [37, 74, 111, 148, 185, 222]),     # 259 > 255 is not a split point: 7 units
    (128, 2, list(range(2, 256, 2))),
])
def test_combine_keeps_every_step_th(orc, c0, target, step, kept):
    """Sec. 3.3 / reading 10: combining M_in = 256 units to `target` keeps exactly the
    split points whose 1-based number is a multiple of step = ceil(256 / target)."""
    spec, s, p, enc, c = c0
    assert spec.splits == 256 and -(-256 // target) == step
    d1 = orc.Decoder(orc.combine(c, target))
    assert d1.threads == len(kept) + 1
    # Thread t of the combined stream ends at the Imin of its kept split point t.
    ends = [d1.thread_range(t)[1] for t in range(1, d1.threads)]
    assert ends == [enc.split(k).imin for k in kept]
    assert d1.thread_range(d1.threads)[1] == len(s)


# ---------------------------------------------------------------------------
# Special cases
# ---------------------------------------------------------------------------

def test_single_lane_sync_section_is_one_symbol(orc):
    """W = 1 (the non-interleaved case of Sec. 3): a split is (state, offset, index)."""
    s = _rng_symbols(5, 3000, 16)
    p = orc.params(lanes=1, quant_bits=8, alphabet=16)
    enc = orc.encode(s, p, 8)
    assert enc.threads == 8
    for k in range(1, enc.threads):
        sp = enc.split(k)
        assert sp.imax == sp.imin
    assert np.array_equal(orc.Decoder(enc.container()).all(), s)


def test_one_thread_equals_serial(orc):
    s = _rng_symbols(6, 5000, 200)
    enc = orc.encode(s, orc.params(lanes=32, quant_bits=10), 1)
    d = orc.Decoder(enc.container())
    assert d.threads == 1 and orc.info(enc.container()).metadata_bytes == 0
    assert np.array_equal(d.all(), d.serial())


@pytest.mark.parametrize("N", [0, 1, 5, 31])
def test_fewer_symbols_than_lanes(orc, N):
    s = _rng_symbols(7, N, 10)
    enc = orc.encode(s, orc.params(lanes=32, quant_bits=8, alphabet=10), 16)
    assert enc.threads == 1
    d = orc.Decoder(enc.container())
    assert np.array_equal(d.all(), s)
    assert np.array_equal(d.serial(), s)


def test_wide_symbols(orc):
    s = _rng_symbols(8, 20000, 4096, np.uint16)
    p = orc.params(lanes=32, quant_bits=12, symbol_bytes=2, alphabet=4096)
    enc = orc.encode(s, p, 10)
    d = orc.Decoder(enc.container())
    assert d.threads == 10
    assert np.array_equal(d.all(), s) and np.array_equal(d.all(aligned=True), s)


# ---------------------------------------------------------------------------
# Brute force on tiny parameters: every sequence, every single split point
# ---------------------------------------------------------------------------

def _all_single_splits_decode(orc, p, f, s):
    enc = orc.encode(s, p, 1, freq=f)
    c = enc.container()
    hdr = _fmt.parse(c)
    assert np.array_equal(orc.Decoder(c).serial(), s)
    cands = []
    for k in range(hdr["B"]):
        cand = enc.candidate_at(k)
        if cand is None:
            continue
        cands.append(cand)
        cc = orc.assemble(p, len(s), f, hdr["words"], hdr["final"], [cand.pos],
                          cand.states[None, :], cand.indices[None, :])
        d = orc.Decoder(cc)
        assert np.array_equal(d.all(fill=255), s), (s.tolist(), cand.pos)
        assert np.array_equal(d.all(aligned=True, fill=255), s), (s.tolist(), cand.pos)
    # Every pair of candidates as a two-split set.
    for a, b in itertools.combinations(cands, 2):
        if b.imin < a.imin:
            continue
        cc = orc.assemble(p, len(s), f, hdr["words"], hdr["final"], [a.pos, b.pos],
                          np.stack([a.states, b.states]), np.stack([a.indices, b.indices]))
        assert np.array_equal(orc.Decoder(cc).all(fill=255), s), (s.tolist(), a.pos, b.pos)
    return len(cands)


@pytest.mark.parametrize("lanes,length", [(1, 7), (2, 7), (3, 7)])
def test_brute_force_tiny_parameters(orc, lanes, length):
    """L = 2^4, b = 4, n = 3, alphabet 3: all sequences of the given length."""
    p = orc.params(lanes=lanes, quant_bits=3, alphabet=3, l_bits=4, b_bits=4)
    f = np.array([1, 2, 5], dtype=np.uint32)
    total = 0
    for seq in itertools.product(range(3), repeat=length):
        total += _all_single_splits_decode(orc, p, f, np.array(seq, dtype=np.uint8))
    assert total > 0


def test_brute_force_real_parameters_skewed_binary(orc):
    """32-bit states, L = 2^16, b = 16, n = 12, f = (1, 4095): all binary sequences of length 12."""
    p = orc.params(lanes=2, quant_bits=12, alphabet=2)
    f = np.array([1, 4095], dtype=np.uint32)
    total = 0
    for seq in itertools.product(range(2), repeat=12):
        total += _all_single_splits_decode(orc, p, f, np.array(seq, dtype=np.uint8))
    assert total > 0


# ---------------------------------------------------------------------------
# Conventional partitioning (Sec. 2.3), the comparison baseline
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("lanes", [1, 3, 32])
def test_partitioned_closed_form_words(orc, lanes):
    """f = 1 at n = 8: every sub-sequence restarts from L, so its words are the
    closed form of its own symbols (first symbol alone, then byte pairs)."""
    N = 37 * lanes + 5
    s = _rng_symbols(50 + lanes, N, 256)
    p = orc.params(lanes=lanes, quant_bits=8, alphabet=256)
    c = _fmt.parse_partitioned(orc.encode_partitioned(s, p, 4, freq=np.ones(256, dtype=np.uint32)))
    S = c["S"]
    assert S % lanes == 0 and c["P"] == -(-N // S) and S == -(-(-(-N // 4)) // lanes) * lanes
    for q in range(c["P"]):
        sub = s[q * S: min(N, (q + 1) * S)]
        expect = []
        groups = -(-len(sub) // lanes)
        for m in range(1, groups, 2):
            for j in range(lanes):
                if m * lanes + j >= len(sub):
                    continue
                local = sub[j::lanes]
                expect.append(int(local[0]) if m == 1 else (int(local[m - 2]) << 8) | int(local[m - 1]))
        assert c["part_words"][q].tolist() == expect, f"sub-sequence {q}"
    assert np.array_equal(orc.Decoder(orc.encode_partitioned(s, p, 4, freq=np.ones(256, np.uint32))).serial(), s)


def test_partitioned_one_part_is_the_plain_stream(orc, c0):
    """One sub-sequence is plain W-way interleaved rANS: the same words and final
    states as the Recoil container with one decode unit."""
    _, s, p, _, _ = c0
    plain = _fmt.parse(orc.encode(s, p, 1).container())
    part = _fmt.parse_partitioned(orc.encode_partitioned(s, p, 1))
    assert part["P"] == 1 and part["S"] >= len(s)
    assert np.array_equal(part["words"], plain["words"])
    assert np.array_equal(part["final"][0], plain["final"])


def test_partitioned_parts_are_independent_streams(orc, c0):
    """Each sub-sequence's words and final states are those of a one-unit encoding
    of that sub-sequence alone with the same table (nothing carries across)."""
    _, s, p, _, _ = c0
    f = _fmt_table(orc, s, p)
    c = _fmt.parse_partitioned(orc.encode_partitioned(s, p, 7, freq=f))
    S = c["S"]
    for q in range(c["P"]):
        alone = _fmt.parse(orc.encode(s[q * S: (q + 1) * S], p, 1, freq=f).container())
        assert np.array_equal(c["part_words"][q], alone["words"]) and np.array_equal(c["final"][q], alone["final"])


def _fmt_table(orc, s, p):
    counts = np.bincount(s, minlength=p.alphabet).astype(np.uint64)
    return orc.quantize(counts, p.quant_bits)


@pytest.mark.parametrize("lanes,N,P", [(1, 1000, 13), (3, 1001, 7), (32, 100_001, 64), (32, 100_001, 5000),
                                       (32, 20, 4), (64, 64 * 50, 50), (64, 64 * 50 + 1, 50)])
def test_partitioned_round_trip(orc, lanes, N, P):
    s = synth.draw_symbols(synth.zipf_pmf(256, 1.1), 60 + lanes + P, N, np.uint8)
    p = orc.params(lanes=lanes, quant_bits=11)
    cont = orc.encode_partitioned(s, p, P)
    d = orc.Decoder(cont)
    S = _fmt.parse_partitioned(cont)["S"]
    assert d.threads == -(-N // S) <= P and S % lanes == 0
    assert np.array_equal(d.serial(), s) and np.array_equal(d.all(workers=3), s)
    for t in (1, d.threads):
        lo, hi = d.thread_range(t)
        assert (lo, hi) == ((t - 1) * S, min(N, t * S))
    with pytest.raises(orc.OracleError):
        orc.combine(cont, 2)


def test_partitioned_overhead_per_part(orc):
    """The cost of partitioning grows linearly with the number of sub-sequences; at
    W = 32 each extra sub-sequence adds about 93-103 bytes in the paper's
    Conventional Large variation (Tables 5-6: +203..224 KB over 2176 partitions)."""
    s = synth.draw_symbols(synth.laplace_pmf(256, 128, 16), 77, 1 << 22, np.uint8)
    p = orc.params(lanes=32, quant_bits=11)
    base = len(orc.encode_partitioned(s, p, 1))
    per = []
    for P in (256, 2176):
        per.append((len(orc.encode_partitioned(s, p, P)) - base) / (P - 1))
    assert all(85 <= v <= 115 for v in per), per
    assert abs(per[0] - per[1]) / per[1] < 0.1


# ---------------------------------------------------------------------------
# Adaptive coding (Sec. 3.1, third advantage of storing symbol indices)
# ---------------------------------------------------------------------------

def test_adaptive_one_table_is_static(orc, c0):
    """One table and an all-zero index: the same words, final states and metadata
    as the static container; only the magic and the table count differ."""
    _, s, p, _, _ = c0
    f = _fmt_table(orc, s, p)
    static = orc.encode(s, p, 64, freq=f).container()
    adapt = orc.encode_adaptive(s, p, f[None, :], np.zeros(len(s), np.uint8), 64).container()
    assert adapt[:4] == b"RCA1" and static[:4] == b"RCL1"
    assert adapt[4:44] == static[4:44] and int.from_bytes(adapt[44:48], "little") == 1
    assert adapt[48:] == static[48:]


def test_adaptive_two_table_code_length(orc):
    """Table 0: 256 symbols of f = 1 at n = 8 (each symbol is x -> 256 x + s, 8 bits);
    table 1: f = 128 for symbols 0 and 1 (x -> 2 x - (x mod 128) + F, 1 bit). With the
    index choosing per symbol, the code length is 8 bits per table-0 symbol plus 1
    bit per table-1 symbol, within log2(e) 2^(n-1) / L per step."""
    N, W = 4096, 1
    tidx = (synth.splitmix64(31, 0, N) % np.uint64(2)).astype(np.uint8)
    s = _rng_symbols(32, N, 256)
    s[tidx == 1] &= 1
    t0 = np.ones(256, np.uint32)
    t1 = np.zeros(256, np.uint32)
    t1[:2] = 128
    p = orc.params(lanes=W, quant_bits=8)
    enc = orc.encode_adaptive(s, p, np.stack([t0, t1]), tidx, 1)
    c = enc.container()
    B = int.from_bytes(c[24:32], "little")
    table_bytes = int.from_bytes(c[36:40], "little")
    final = np.frombuffer(c[48 + table_bytes: 48 + table_bytes + 4 * W], dtype="<u4")
    total = 16 * B + sum(math.log2(int(x)) for x in final) - 16 * W
    ideal = 8 * int((tidx == 0).sum()) + int((tidx == 1).sum())
    assert abs(total - ideal) <= N * 1.4427 * 128 / 2.0 ** 16
    d = orc.Decoder(c)
    d.set_table_index(tidx)
    assert np.array_equal(d.serial(), s)


def test_adaptive_round_trip_threads_combine_and_wrong_index(orc):
    """Per-symbol tables chosen from a seeded index: serial and per-split decoding,
    combining, and a decoder given a different index does not reproduce the input."""
    N, T, A = 150_001, 6, 64
    tidx = (synth.splitmix64(7, 0, N) % np.uint64(T)).astype(np.uint8)
    tabs = np.stack([orc.quantize((synth.laplace_pmf(A, A / 2, 0.7 + 3 * t) * 1e6 + 1).astype(np.uint64), 10)
                     for t in range(T)])
    s = np.zeros(N, np.uint8)
    for t in range(T):
        m = tidx == t
        s[m] = synth.draw_symbols(synth.laplace_pmf(A, A / 2, 0.7 + 3 * t), 40 + t, int(m.sum()), np.uint8)
    for W in (32, 64):
        p = orc.params(lanes=W, quant_bits=10, alphabet=A)
        c = orc.encode_adaptive(s, p, tabs, tidx, 100).container()
        d = orc.Decoder(c)
        with pytest.raises(orc.OracleError):
            d.serial()                                     # the index is required
        d.set_table_index(tidx)
        assert d.threads == 100
        assert np.array_equal(d.serial(), s) and np.array_equal(d.all(aligned=True, workers=3), s)
        for target in (7, 1):
            dc = orc.Decoder(orc.combine(c, target))
            dc.set_table_index(tidx)
            assert np.array_equal(dc.all(), s)
        wrong = tidx.copy()
        wrong[::5] = (wrong[::5] + 1) % T
        dw = orc.Decoder(c)
        dw.set_table_index(wrong)
        try:
            assert not np.array_equal(dw.serial(), s)
        except orc.OracleError:
            pass


@pytest.mark.parametrize("lanes", [1, 2])
def test_adaptive_brute_force_tiny(orc, lanes):
    """L = 2^4, b = 4, n = 3, two tables over 3 symbols: every sequence of length 6
    with two index patterns, encoded with 1..3 decode units, decodes exactly."""
    p = orc.params(lanes=lanes, quant_bits=3, alphabet=3, l_bits=4, b_bits=4)
    tabs = np.array([[1, 2, 5], [6, 1, 1]], dtype=np.uint32)
    for seq in itertools.product(range(3), repeat=6):
        s = np.array(seq, dtype=np.uint8)
        for pat in (np.array([0, 1, 1, 0, 1, 0], np.uint8), np.array([1, 1, 1, 0, 0, 0], np.uint8)):
            for threads in (1, 2, 3):
                c = orc.encode_adaptive(s, p, tabs, pat, threads).container()
                d = orc.Decoder(c)
                d.set_table_index(pat)
                assert np.array_equal(d.serial(), s)
                assert np.array_equal(d.all(fill=255), s) and np.array_equal(d.all(aligned=True, fill=255), s)
