"""GPU parity: librecoil's HIP decoder against the seeded input symbols.

Recoil is lossless, so the expected output of a decode is the symbol sequence
that was encoded (drawn by the seeded generators in `synth`). Containers come
either from librecoil's encoder (checked byte-identical to the oracle's in the
CPU tests) or directly from the oracle (arbitrary split sets). Every output is
compared element by element, bit-exact; the output buffer is pre-filled with
two different patterns so that a symbol left unwritten is caught.
"""

import itertools
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2306_12141_amd as m
    return m


def gpu_decode(rc, blob, poison=(0xA5, 0x5A), **tuning):
    """Decode twice, into buffers pre-filled with two patterns; both must agree."""
    plan = rc.Plan(blob)
    if tuning:
        plan.set_tuning(**tuning)
    ws = plan.allocate_workspace()
    plan.upload(ws)
    outs = []
    for pv in poison:
        out = plan.allocate_output()
        out.fill_(pv)
        err = torch.zeros(1, dtype=torch.int32, device="cuda")
        plan.decode(ws, out, err)
        torch.cuda.synchronize()
        assert int(err.item()) == 0
        outs.append(plan.symbols_of(out))
    assert np.array_equal(outs[0], outs[1]), "some symbols were not written"
    return outs[0]


def _syms(seed, n, A, dtype=np.uint8, skew=None):
    if skew is None:
        return (synth.splitmix64(seed, 0, n) % np.uint64(A)).astype(dtype)
    return synth.draw_symbols(synth.zipf_pmf(A, skew), seed, n, dtype)


def test_c0_laplace_1mib(rc, orc):
    spec = synth.c0_spec()
    s = spec.generate()
    _say("case c0", spec)
    blob = rc.encode(s, lanes=32, quant_bits=11, splits=256)
    assert blob.splits == 256
    out = gpu_decode(rc, blob)
    assert np.array_equal(out, s)


@pytest.mark.parametrize("target", [128, 100, 17, 2, 1])
def test_c0_combined(rc, target):
    spec = synth.c0_spec()
    s = spec.generate()
    _say("case c0 combined", target)
    blob = rc.encode(s, lanes=32, quant_bits=11, splits=256).combine(target)
    assert np.array_equal(gpu_decode(rc, blob), s)


CASES = [
    # (lanes, n, symbol dtype, alphabet, N, splits, zipf exponent or None)
    (32, 11, np.uint8, 256, 100_000, 37, 1.1),
    (64, 11, np.uint8, 256, 100_000, 37, 1.1),
    (32, 12, np.uint8, 256, 300_001, 64, 0.8),
    (64, 12, np.uint8, 256, 300_001, 64, 1.5),
    (32, 10, np.uint8, 200, 77_777, 9, None),
    (32, 12, np.uint16, 4096, 120_003, 20, 1.0),
    (64, 12, np.uint16, 4096, 120_003, 20, 1.3),
    (32, 12, np.uint16, 4096, 50_000, 5, None),
    (32, 8, np.uint8, 3, 40_000, 30, 2.5),
    (64, 8, np.uint8, 2, 40_000, 30, 3.0),
    (32, 11, np.uint8, 256, 31, 4, None),       # N < W: one unit
    (64, 11, np.uint8, 256, 65, 4, None),       # partial last group
    (32, 11, np.uint8, 256, 1, 1, None),
]


@pytest.mark.parametrize("waves", [0, 16])
@pytest.mark.parametrize("ci", range(len(CASES)), ids=[f"W{c[0]}_n{c[1]}_{np.dtype(c[2]).name}_N{c[4]}_M{c[5]}" for c in CASES])
def test_streams(rc, ci, waves):
    """Each stream shape with the default launch shape (one wave per workgroup for
    these few units) and with 16-wave workgroups."""
    W, n, dt, A, N, M, z = CASES[ci]
    _say("case", CASES[ci], waves)
    s = _syms(1000 + ci, N, A, dt, z)
    blob = rc.encode(s, lanes=W, quant_bits=n, splits=M, alphabet=A)
    tuning = dict(waves=16, chunk_groups=8 if dt == np.uint8 else 4) if waves else {}
    assert np.array_equal(gpu_decode(rc, blob, **tuning), s)


@pytest.mark.parametrize("W,N,dt,k", [(32, 200, np.uint8, 1), (32, 1392, np.uint8, 1), (32, 1392, np.uint8, 3),
                                      (64, 1392, np.uint16, 1), (64, 5000, np.uint8, 1), (64, 5000, np.uint8, 4)])
def test_more_units_than_groups(rc, W, N, dt, k):
    """A small stream cut finer than its symbol groups (several split points in one
    group, some units empty), decoded from the encoder's blob and from its container."""
    A = 256 if dt == np.uint8 else 4096
    _say("case more units than groups", W, N, np.dtype(dt).name, k)
    s = _syms(77 + W + N, N, A, dt, 1.1)
    blob = rc.encode(s, lanes=W, quant_bits=12, splits=400, alphabet=A)
    assert blob.info.splits > -(-N // W)
    tuning = dict(chunk_groups=8 if dt == np.uint8 else 4, units_per_run=k)
    assert np.array_equal(gpu_decode(rc, blob, **tuning), s)
    assert np.array_equal(gpu_decode(rc, rc.Blob.from_bytes(blob.to_bytes()), **tuning), s)


RUN_CASES = [
    # (lanes, n, symbol dtype, alphabet, N, splits, zipf exponent or None)
    (32, 11, np.uint8, 256, 200_003, 29, 1.1),
    (64, 12, np.uint8, 256, 300_001, 23, 1.3),
    (32, 12, np.uint16, 4096, 120_003, 11, 1.0),
    (64, 12, np.uint16, 4096, 90_001, 7, None),
]


@pytest.mark.parametrize("k", [2, 3, 5, 10_000])
@pytest.mark.parametrize("ci", range(len(RUN_CASES)), ids=[f"W{c[0]}_{np.dtype(c[2]).name}_M{c[5]}" for c in RUN_CASES])
def test_units_per_run(rc, ci, k):
    """Runs of k consecutive units decoded as one (the last run ragged; k >= M is
    the whole stream as one unit, i.e. the serial interleaved decoder)."""
    W, n, dt, A, N, M, z = RUN_CASES[ci]
    _say("case runs", RUN_CASES[ci], k)
    s = _syms(2000 + ci, N, A, dt, z)
    blob = rc.encode(s, lanes=W, quant_bits=n, splits=M, alphabet=A)
    assert np.array_equal(gpu_decode(rc, blob, waves=16, chunk_groups=8 if dt == np.uint8 else 4, units_per_run=k), s)


def test_units_per_run_shape(rc):
    """The shape query reports the runs a launch decodes; 0 chooses at most one run per unit slot."""
    s = _syms(77, 1 << 20, 256, np.uint8, 1.1)
    blob = rc.encode(s, lanes=64, quant_bits=12, splits=4096)
    M = blob.splits
    assert M > 1000
    plan = rc.Plan(blob)
    plan.set_tuning(waves=16, chunk_groups=8, units_per_run=3)
    sh = plan.shape()
    assert sh.units_per_run == 3 and sh.runs == -(-M // 3) and sh.waves_per_block == 16
    plan.set_tuning(waves=16, chunk_groups=8, units_per_run=0)
    sh = plan.shape()
    assert sh.units_per_run >= 1 and sh.runs == -(-M // sh.units_per_run)
    assert sh.runs <= sh.blocks * sh.waves_per_block           # W = 64: one unit slot per wave


@pytest.mark.parametrize("W,splits,dt", [(32, 256, np.uint8), (64, 900, np.uint8), (32, 3000, np.uint16),
                                          (64, 4096, np.uint8)])
def test_waves_per_workgroup(rc, W, splits, dt):
    """The default shape puts one wave in each workgroup when the decode has no more
    wave-sized pieces of work than the chip has SIMDs, 8 when 16-wave workgroups would
    not reach every CU, 16 otherwise; explicit 1, 8 and 16 waves decode the same symbols."""
    _say("case waves per workgroup", W, splits, np.dtype(dt).name)
    A = 256 if dt == np.uint8 else 4096
    s = _syms(91 + splits, 1 << 20, A, dt, 1.1)
    blob = rc.encode(s, lanes=W, quant_bits=12, splits=splits, alphabet=A)
    plan = rc.Plan(blob)
    sh = plan.shape()
    pieces = -(-sh.runs // sh.units_per_wave)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    assert sh.waves_per_block == (1 if pieces <= 4 * cus else 8 if pieces < 16 * cus else 16)
    k = 8 if dt == np.uint8 else 4
    assert np.array_equal(gpu_decode(rc, blob), s)
    for w in (1, 8, 16):
        assert np.array_equal(gpu_decode(rc, blob, waves=w, chunk_groups=k), s)


@pytest.mark.parametrize("N,M", [((1 << 22) + 77, 20_000), ((1 << 20) + 5, 300), (70_001, 12)])
def test_w32_byte_symbols_every_shape(rc, N, M):
    """32-lane units store byte symbols one dword per four groups (a byte transpose
    across each quad of lanes): every launch shape (1, 8 and 16 waves; 4- and 8-group
    super-steps; runs of 1, 3 and automatic length; one unit or a pair per wave)
    decodes the input, ragged last group included."""
    s = _syms(4400 + M, N, 256, np.uint8, 1.1)
    blob = rc.encode(s, lanes=32, quant_bits=12, splits=M, alphabet=256)
    per_wave = set()
    for w, k, r in itertools.product((1, 8, 16), (4, 8), (0, 1, 3)):
        _say("case w32 byte symbols", N, M, w, k, r)
        plan = rc.Plan(blob)
        plan.set_tuning(waves=w, chunk_groups=k, units_per_run=r)
        per_wave.add(plan.shape().units_per_wave)
        assert np.array_equal(gpu_decode(rc, blob, waves=w, chunk_groups=k, units_per_run=r), s)
    if M == 20_000:
        assert 2 in per_wave    # 20000 runs of one unit exceed the resident waves: the pair kernel
    if M == 12:
        assert per_wave == {1}


def test_plan_autotune(rc):
    """The single-stream autotuner leaves a valid shape on the plan, the decode with it
    is exact, and a second plan of the same shape is served from the cache."""
    s = _syms(55, 1 << 20, 256, np.uint8, 1.1)
    blob = rc.encode(s, lanes=64, quant_bits=12, splits=2048)
    plan = rc.Plan(blob)
    ws = plan.allocate_workspace()
    plan.upload(ws)
    out = plan.allocate_output()
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    best, ms = plan.autotune(ws, out, err, reps=2)
    assert best.waves in (1, 8, 16) and best.chunk_groups in (4, 8) and best.units_per_run in (0, 1, 2, 4)
    assert ms > 0
    out.fill_(0x3C)
    err.zero_()
    plan.decode(ws, out, err)
    torch.cuda.synchronize()
    assert int(err.item()) == 0 and np.array_equal(plan.symbols_of(out), s)
    plan2 = rc.Plan(blob)
    best2, ms2 = plan2.autotune(ws, out, err, reps=2)
    assert ms2 == -1.0 and (best2.waves, best2.chunk_groups, best2.units_per_run) == \
        (best.waves, best.chunk_groups, best.units_per_run)


def test_random_split_sets_runs(rc, orc):
    """Irregular oracle-built split sets decoded in runs of 2 and 3 units."""
    from tests import _fmt
    W, N = 64, 30_000
    s = _syms(98, N, 256, np.uint8, 1.2)
    p = orc.params(lanes=W, quant_bits=12)
    f = orc.quantize(np.bincount(s, minlength=256).astype(np.uint64), 12)
    enc = orc.encode(s, p, 1, freq=f)
    hdr = _fmt.parse(enc.container())
    rng = np.random.default_rng(6)
    cands = []
    for k in rng.choice(hdr["B"], size=300, replace=False):
        c = enc.candidate_at(int(k))
        if c is not None:
            cands.append(c)
    cands.sort(key=lambda c: c.pos)
    for trial in range(4):
        pick = sorted(rng.choice(len(cands), size=min(len(cands), 4 + 7 * trial), replace=False))
        chosen = [cands[i] for i in pick]
        chosen = [c for i, c in enumerate(chosen) if all(c.imin >= d.imin for d in chosen[:i])]
        cont = orc.assemble(p, N, f, hdr["words"], hdr["final"], [c.pos for c in chosen],
                            np.stack([c.states for c in chosen]), np.stack([c.indices for c in chosen]))
        for k in (2, 3):
            assert np.array_equal(gpu_decode(rc, rc.Blob.from_bytes(cont), chunk_groups=8, units_per_run=k), s)


@pytest.mark.parametrize("W", [32, 64])
def test_c1_full_size(rc, W):
    """The 256 MiB Zipf(1.1) stream with 65536 splits in the launch configuration
    the benchmark times (default tuning), and with every split point used."""
    spec = synth.c1_spec(W)
    _say("case c1 full", W)
    s = spec.generate()
    blob = rc.encode(s, lanes=W, quant_bits=spec.quant_bits, splits=spec.splits)
    assert blob.splits == spec.splits
    plan = rc.Plan(blob)
    ws = plan.allocate_workspace()
    plan.upload(ws)
    for tuning in ({}, {"waves": 16, "chunk_groups": 8, "units_per_run": 1}):
        if tuning:
            plan.set_tuning(**tuning)
        out = plan.allocate_output()
        out.fill_(0xA5)
        err = torch.zeros(1, dtype=torch.int32, device="cuda")
        plan.decode(ws, out, err)
        torch.cuda.synchronize()
        assert int(err.item()) == 0
        got = plan.symbols_of(out)
        assert np.array_equal(got, s), (tuning, int(np.flatnonzero(got != s)[0]))
        del out


def test_single_symbol_stream(rc):
    s = np.full(10_000, 7, dtype=np.uint8)
    for n in (8, 12):
        blob = rc.encode(s, lanes=32, quant_bits=n, splits=4)
        assert np.array_equal(gpu_decode(rc, blob), s)


def test_empty_stream(rc):
    s = np.zeros(0, dtype=np.uint8)
    blob = rc.encode(s, lanes=32, quant_bits=8, splits=1)
    assert gpu_decode(rc, blob).size == 0


@pytest.mark.parametrize("W", [32, 64])
def test_every_single_split_point(rc, orc, W):
    """Every usable split word of a small stream as a lone split (oracle-built containers)."""
    from tests import _fmt
    N = 40 * W + 5
    s = _syms(3 + W, N, 4, np.uint8, 1.2)
    p = orc.params(lanes=W, quant_bits=10, alphabet=4)
    f = orc.quantize(np.bincount(s, minlength=4).astype(np.uint64), 10)
    enc = orc.encode(s, p, 1, freq=f)
    hdr = _fmt.parse(enc.container())
    n_cand = 0
    for k in range(hdr["B"]):
        cand = enc.candidate_at(k)
        if cand is None:
            continue
        n_cand += 1
        c = orc.assemble(p, N, f, hdr["words"], hdr["final"], [cand.pos], cand.states[None, :],
                         cand.indices[None, :])
        blob = rc.Blob.from_bytes(c)
        assert np.array_equal(gpu_decode(rc, blob), s), k
    assert n_cand > 0


def test_random_split_sets(rc, orc):
    from tests import _fmt
    W, N = 32, 20_000
    s = _syms(99, N, 256, np.uint8, 1.1)
    p = orc.params(lanes=W, quant_bits=11)
    f = orc.quantize(np.bincount(s, minlength=256).astype(np.uint64), 11)
    enc = orc.encode(s, p, 1, freq=f)
    hdr = _fmt.parse(enc.container())
    rng = np.random.default_rng(5)
    cands = []
    for k in rng.choice(hdr["B"], size=400, replace=False):
        c = enc.candidate_at(int(k))
        if c is not None:
            cands.append(c)
    cands.sort(key=lambda c: c.pos)
    for trial in range(6):
        pick = sorted(rng.choice(len(cands), size=min(len(cands), 3 + 9 * trial), replace=False))
        chosen = [cands[i] for i in pick]
        # Synchronisation points must be monotone (the container validator enforces it).
        chosen = [c for i, c in enumerate(chosen) if all(c.imin >= d.imin for d in chosen[:i])]
        cont = orc.assemble(p, N, f, hdr["words"], hdr["final"], [c.pos for c in chosen],
                            np.stack([c.states for c in chosen]), np.stack([c.indices for c in chosen]))
        assert np.array_equal(gpu_decode(rc, rc.Blob.from_bytes(cont)), s)


def test_corrupt_offset_sets_error_word(rc, orc):
    """A container that passes host validation but makes unit 0 run out of words."""
    from tests import _fmt
    W, N = 32, 4000
    s = _syms(17, N, 256, np.uint8, 1.1)
    p = orc.params(lanes=W, quant_bits=11)
    f = orc.quantize(np.bincount(s, minlength=256).astype(np.uint64), 11)
    enc = orc.encode(s, p, 1, freq=f)
    hdr = _fmt.parse(enc.container())
    cand = next(c for c in (enc.candidate_at(k) for k in range(hdr["B"] - 1, 0, -1)) if c is not None)
    # Claim the split word is word 0: the unit starts with one word and needs many.
    cont = orc.assemble(p, N, f, hdr["words"], hdr["final"], [0], cand.states[None, :], cand.indices[None, :])
    blob = rc.Blob.from_bytes(cont)
    plan = rc.Plan(blob)
    ws = plan.allocate_workspace()
    plan.upload(ws)
    out = plan.allocate_output()
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    plan.decode(ws, out, err)
    torch.cuda.synchronize()
    assert int(err.item()) & 1


def _run_on_windows(rec, shape, K):
    """Groups that each run may store a second time (the run-on below its own lowest
    group): after synchronisation a run decodes whole K-group super-steps up to its
    pair's longest run, so at most (kmax - steps) + K - 1 groups below its glo."""
    M, k, S = len(rec), shape.units_per_run, shape.units_per_wave
    runs = []
    for r in range(shape.runs):
        lo, hi = r * k, min(r * k + k, M) - 1
        top, glo = int(rec[hi][1]), int(rec[lo][3])
        runs.append((glo, max(0, top + 1 - glo)))
    wins = []
    for r, (glo, steps) in enumerate(runs):
        mates = runs[r - r % S: r - r % S + S]
        kmax = max(st for _, st in mates)
        wins.append((max(0, glo - (kmax - steps) - (K - 1)), glo - 1))
    return wins


@pytest.mark.parametrize("case", ["c0", "w32_pairs", "w64", "u16_pairs", "small_units"])
def test_write_counts(rc, case):
    """Every symbol is stored at least once, and a second store happens only in the
    run-on window of the run above (Sec. 4.1.3 ownership plus the run-on)."""
    if case == "c0":
        spec = synth.c0_spec()
        s, W, n, A, M, kw = spec.generate(), 32, spec.quant_bits, 256, spec.splits, {}
    elif case == "w32_pairs":
        s, W, n, A, M, kw = _syms(71, 1 << 23, 256, skew=1.1), 32, 12, 256, 32768, {"units_per_run": 1}
    elif case == "w64":
        s, W, n, A, M, kw = _syms(72, 1 << 23, 256, skew=1.1), 64, 12, 256, 16384, {}
    elif case == "u16_pairs":
        s, W, n, A, M, kw = _syms(73, (1 << 22) + 77, 4096, np.uint16, 1.05), 32, 12, 4096, 32768, {}
    else:
        s, W, n, A, M, kw = _syms(74, 90_001, 256, skew=1.2), 32, 11, 256, 4000, {"units_per_run": 3}
    blob = rc.encode(s, lanes=W, quant_bits=n, splits=M, alphabet=A)
    plan = rc.Plan(blob)
    K = 8 if s.dtype == np.uint8 else 4
    if kw:
        plan.set_tuning(chunk_groups=K, **kw)
    shape = plan.shape()
    ws = plan.allocate_workspace()
    plan.upload(ws)
    out = plan.allocate_output()
    out.fill_(0x6B)
    counts = torch.zeros(len(s), dtype=torch.int32, device="cuda")
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    plan.decode_count_writes(ws, out, counts, err)
    torch.cuda.synchronize()
    assert int(err.item()) == 0
    assert np.array_equal(plan.symbols_of(out), s)
    c = counts.cpu().numpy()
    assert c.min() >= 1, f"{int((c == 0).sum())} symbols never stored"
    allowed = np.zeros(-(-len(s) // W), dtype=np.int64)
    for lo, hi in _run_on_windows(plan.units(), shape, K):
        if hi >= lo:
            allowed[lo:hi + 1] += 1
    extra = c.astype(np.int64) - 1
    limit = np.repeat(allowed, W)[: len(s)]
    bad = np.nonzero(extra > limit)[0]
    assert bad.size == 0, f"symbol {bad[0]} stored {c[bad[0]]} times (group {bad[0] // W}, allowed {limit[bad[0]]})"
    _say(f"{case}: runs {shape.runs} x {shape.units_per_run} units, {shape.units_per_wave} per wave; "
         f"stored twice {int((c > 1).sum())} of {len(s)} ({(c > 1).mean():.4%})")


@pytest.mark.parametrize("W,N,P,dt", [(32, 1_000_003, 4096, np.uint8), (64, 1 << 20, 512, np.uint8),
                                      (32, 300_001, 20_000, np.uint16), (64, 64 * 10_000, 10_000, np.uint16),
                                      (32, 5_000, 1, np.uint8), (32, 77, 9, np.uint8)])
def test_partitioned_streams(rc, orc, W, N, P, dt):
    """The conventional baseline (Sec. 2.3) on the same kernels: every unit starts from
    its sub-sequence's final states. Checked against the input symbols, and every
    symbol is stored exactly once (no synchronisation, no run-on)."""
    A = 256 if dt == np.uint8 else 4096
    s = _syms(900 + P, N, A, dt, skew=1.1)
    n = 12
    blob = rc.encode_partitioned(s, lanes=W, quant_bits=n, partitions=P, alphabet=A)
    assert blob.to_bytes() == orc.encode_partitioned(
        s, orc.params(lanes=W, quant_bits=n, symbol_bytes=np.dtype(dt).itemsize, alphabet=A), P)
    assert np.array_equal(gpu_decode(rc, blob), s)
    plan = rc.Plan(blob)
    assert plan.shape().units_per_run == 1
    ws = plan.allocate_workspace()
    plan.upload(ws)
    out = plan.allocate_output()
    counts = torch.zeros(N, dtype=torch.int32, device="cuda")
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    plan.decode_count_writes(ws, out, counts, err)
    torch.cuda.synchronize()
    assert int(err.item()) == 0
    assert np.array_equal(plan.symbols_of(out), s)
    assert int(counts.min().item()) == 1 and int(counts.max().item()) == 1


@pytest.mark.parametrize("W,n,T,A,nbits,M,run", [(32, 2_000_003, 16, 64, 9, 512, 0), (64, 1 << 21, 8, 64, 10, 300, 0),
                                                (32, 1 << 21, 16, 64, 9, 4096, 1), (32, 1 << 22, 4, 256, 12, 20000, 0),
                                                (64, 100_001, 2, 128, 11, 1000, 3), (32, 70, 16, 64, 9, 3, 0)])
def test_adaptive_streams(rc, orc, W, n, T, A, nbits, M, run):
    """Adaptive coding (Sec. 3.1): every symbol decoded with the table its index names.
    Containers byte-identical to the oracle's; outputs equal the input symbols, also
    combined; a wrong index gives a different output."""
    pmfs, tidx, s = synth.adaptive_stream(700 + T + W, n, T, A)
    tabs = np.stack([orc.quantize((pmf * (1 << 30)).astype(np.uint64) + 1, nbits) for pmf in pmfs])
    blob = rc.encode_adaptive(s, tabs, tidx, lanes=W, quant_bits=nbits, splits=M, alphabet=A)
    assert blob.to_bytes() == orc.encode_adaptive(s, orc.params(lanes=W, quant_bits=nbits, alphabet=A), tabs, tidx,
                                                  M).container()
    d_tidx = torch.from_numpy(tidx).to("cuda")
    for b in (blob, blob.combine(max(1, M // 7))):
        plan = rc.Plan(b)
        if run:
            plan.set_tuning(chunk_groups=4, units_per_run=run)
        ws = plan.allocate_workspace()
        plan.upload(ws)
        for poison in (0xA5, 0x5A):
            out = plan.allocate_output()
            out.fill_(poison)
            err = torch.zeros(1, dtype=torch.int32, device="cuda")
            plan.decode_adaptive(ws, d_tidx, out, err)
            torch.cuda.synchronize()
            assert int(err.item()) == 0
            assert np.array_equal(plan.symbols_of(out), s), f"splits {b.splits}"
    if T > 1:
        wrong = tidx.copy()
        wrong[::3] = (wrong[::3] + 1) % T
        out.fill_(0)
        plan.decode_adaptive(ws, torch.from_numpy(wrong).to("cuda"), out, err)
        torch.cuda.synchronize()
        assert not np.array_equal(plan.symbols_of(out), s)
    with pytest.raises(rc.RecoilError):
        plan.decode(ws, out, err)                   # the index is required


WIDE_CASES = [
    # (lanes, n, symbol dtype, alphabet, N, splits, zipf exponent or None): 13 <= n <= 16
    (32, 16, np.uint8, 256, (1 << 20) + 5, 64, 1.1),
    (64, 16, np.uint8, 256, 300_001, 37, 0.9),
    (32, 13, np.uint8, 256, 200_000, 20, 1.2),
    (64, 14, np.uint8, 200, 150_000, 9, None),
    (32, 16, np.uint8, 256, 100_000, 12, None),      # uniform: every f = 256, no start inside a bucket
    (32, 16, np.uint8, 2, 40_000, 30, 3.0),
    (32, 15, np.uint16, 4096, 200_003, 30, 1.0),
    (64, 16, np.uint16, 4096, 120_003, 20, 1.3),
    (32, 13, np.uint16, 4096, 100_000, 16, None),    # f = 2: eight starts in every bucket
    (32, 16, np.uint8, 256, 31, 4, None),            # N < W
    (64, 16, np.uint8, 256, 65, 4, None),
]


@pytest.mark.parametrize("ci", range(len(WIDE_CASES)),
                         ids=[f"W{c[0]}_n{c[1]}_{np.dtype(c[2]).name}_N{c[4]}_M{c[5]}" for c in WIDE_CASES])
def test_wide_tables(rc, ci):
    """13 <= n <= 16: the two-level LDS table (16-slot buckets, per-symbol entries)
    with the default shape, 8-group super-steps, one unit per run, and combined."""
    W, n, dt, A, N, M, z = WIDE_CASES[ci]
    _say("case wide", WIDE_CASES[ci])
    s = _syms(6000 + ci, N, A, dt, z)
    blob = rc.encode(s, lanes=W, quant_bits=n, splits=M, alphabet=A)
    assert np.array_equal(gpu_decode(rc, blob), s)
    assert np.array_equal(gpu_decode(rc, blob, waves=16, chunk_groups=8), s)
    assert np.array_equal(gpu_decode(rc, blob, waves=8, chunk_groups=4, units_per_run=1), s)
    if M > 2:
        assert np.array_equal(gpu_decode(rc, blob.combine(M // 3)), s)


@pytest.mark.parametrize("W", [32, 64])
def test_wide_full_size(rc, W):
    """The 256 MiB Zipf(1.1) stream of the headline workload, coded at n = 16."""
    spec = synth.c1_spec(W)
    s = spec.generate()
    _say("case wide full", W)
    blob = rc.encode(s, lanes=W, quant_bits=16, splits=spec.splits)
    assert np.array_equal(gpu_decode(rc, blob), s)


def test_wide_partitioned_and_packed(rc):
    """n = 16 with the other plan kinds: conventional sub-sequences decoded through the
    two-level table, and a packed plan (records unpacked on the device)."""
    s = _syms(6100, 1_000_003, 256, np.uint8, 1.1)
    _say("case wide partitioned / packed")
    part = rc.encode_partitioned(s, lanes=32, quant_bits=16, partitions=300)
    assert np.array_equal(gpu_decode(rc, part), s)
    blob = rc.encode(s, lanes=64, quant_bits=16, splits=200)
    for t in (0, 50):
        plan = rc.Plan(blob, packed_target=t)
        ws = plan.allocate_workspace()
        plan.upload(ws)
        out = plan.allocate_output()
        out.fill_(0xA5)
        err = torch.zeros(1, dtype=torch.int32, device="cuda")
        plan.decode(ws, out, err)
        torch.cuda.synchronize()
        assert int(err.item()) == 0
        assert np.array_equal(plan.symbols_of(out), s), f"packed target {t}"


def test_above_2gib_output(rc):
    """The largest outputs: 2^31 + 4099 uint8 symbols (output offsets and symbol
    indices past 2^31), W = 64, 65536 units, the default launch shape."""
    N = (1 << 31) + 4099
    s = synth.draw_symbols(synth.zipf_pmf(256, 1.1), 6200, N, np.uint8)
    _say("case 2 GiB + 4099 symbols")
    blob = rc.encode(s, lanes=64, quant_bits=12, splits=65536)
    assert blob.info.n_words < (1 << 31) - 1024
    assert np.array_equal(gpu_decode(rc, blob), s)
