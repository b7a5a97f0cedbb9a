"""GPU parity of the batched persistent decoder, the per-stream baseline, HIP
graph replays, the autotuner and every launch shape of the single-stream kernel.

Expected outputs are the seeded input symbols of every stream (lossless codec);
comparisons are bit-exact.
"""

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


def _mixed_streams(rc, count=48, seed=77):
    """Small streams covering the batch's variety: uint8/uint16, W 32/64, n 8..12,
    single-symbol and tiny streams."""
    out = []
    for i in range(count):
        spec = synth.mixed_stream_spec(seed, i, 1 << 10, 1 << 19, 4 << 10)
        s = spec.generate()
        lanes = 64 if i % 5 == 4 else 32
        present = int(np.count_nonzero(np.bincount(s, minlength=spec.alphabet)))
        n = max(spec.quant_bits, int(np.ceil(np.log2(max(present, 2)))))
        if i == 7:
            s = np.full(5000, 3, dtype=spec.dtype)         # one symbol only
        if i == 11:
            s = s[:20]                                      # fewer symbols than lanes
        blob = rc.encode(s, lanes=lanes, quant_bits=n, splits=spec.splits, alphabet=spec.alphabet)
        out.append((s, blob))
    return out


@pytest.fixture(scope="module")
def mixed(rc):
    return _mixed_streams(rc)


def _check_all(batch, out, streams):
    for i, (s, _) in enumerate(streams):
        got = batch.symbols_of(out, i, s.dtype)
        assert np.array_equal(got, s), f"stream {i}"


def test_batch_persistent_and_per_stream(rc, mixed):
    from paper_2306_12141_amd.batch import Batch
    batch = Batch([b for _, b in mixed])
    _say("batch items", batch.items, "ws", batch.workspace_bytes)
    ws, out, err = batch.allocate()
    batch.upload(ws)
    out.fill_(0xEE)
    batch.decode(ws, out, err)
    torch.cuda.synchronize()
    assert int(err.item()) == 0
    _check_all(batch, out, mixed)
    out.fill_(0x11)
    batch.decode_per_stream(ws, out, err)
    torch.cuda.synchronize()
    assert int(err.item()) == 0
    _check_all(batch, out, mixed)


@pytest.mark.parametrize("shape", [(16, 4, 1), (16, 4, 2), (8, 4, 4), (8, 8, 1), (8, 8, 8), (16, 8, 2),
                                   (16, 4, 2, 2), (8, 8, 1, 3), (16, 8, 4, 4), (16, 4, 8, 64)])
def test_batch_shapes(rc, mixed, shape):
    from paper_2306_12141_amd._lib import Tuning
    from paper_2306_12141_amd.batch import Batch
    batch = Batch([b for _, b in mixed], Tuning(shape[0], shape[1], shape[2], 0, shape[3] if len(shape) > 3 else 0))
    ws, out, err = batch.allocate()
    batch.upload(ws)
    out.fill_(0x5A)
    batch.decode(ws, out, err)
    torch.cuda.synchronize()
    assert int(err.item()) == 0
    _check_all(batch, out, mixed)


@pytest.mark.parametrize("width", [np.uint8, np.uint16])
def test_batch_one_table_class(rc, mixed, width):
    """A batch whose streams all fall in one decode-table class (the other class's
    launch is skipped), in a graph replayed twice."""
    from paper_2306_12141_amd.batch import Batch
    sel = [(s, b) for s, b in mixed if s.dtype == width]
    assert len(sel) >= 4
    batch = Batch([b for _, b in sel])
    ws, out, err = batch.allocate()
    batch.upload(ws)
    g = batch.graph(ws, out, err)
    for rep in range(2):
        out.fill_(0xA5 if rep else 0x5A)
        g.launch()
        torch.cuda.synchronize()
        assert int(err.item()) == 0
        _check_all(batch, out, sel)


def test_batch_more_units_than_groups(rc):
    """Streams cut finer than their symbol groups (some units empty) in one batch."""
    from paper_2306_12141_amd.batch import Batch
    streams = []
    for i, (W, N, dt) in enumerate([(32, 200, np.uint8), (32, 1392, np.uint8), (64, 1392, np.uint16),
                                    (64, 5000, np.uint8)]):
        A = 256 if dt == np.uint8 else 4096
        s = synth.draw_symbols(synth.zipf_pmf(A, 1.1), 900 + i, N, dt)
        blob = rc.encode(s, lanes=W, quant_bits=12, splits=400, alphabet=A)
        assert blob.info.splits > -(-N // W)
        streams.append((s, blob))
    batch = Batch([b for _, b in streams])
    ws, out, err = batch.allocate()
    batch.upload(ws)
    out.fill_(0x5A)
    batch.decode(ws, out, err)
    torch.cuda.synchronize()
    assert int(err.item()) == 0
    _check_all(batch, out, streams)


def test_graph_replays(rc, mixed):
    """The captured graph replays several times, with eager work in between;
    each replay must equal the eager result."""
    from paper_2306_12141_amd.batch import Batch
    batch = Batch([b for _, b in mixed])
    ws, out, err = batch.allocate()
    batch.upload(ws)
    torch.cuda.synchronize()
    g = batch.graph(ws, out, err)
    for r in range(4):
        out.fill_(r)
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        assert int(err.item()) == 0
        _check_all(batch, out, mixed)
        junk = torch.ones(1 << 20, device="cuda").sum()       # eager work between replays
        torch.cuda.synchronize()
        del junk


def test_autotune(rc, mixed):
    from paper_2306_12141_amd.batch import Batch
    batch = Batch([b for _, b in mixed])
    ws, out, err = batch.allocate()
    batch.upload(ws)
    best, ms = batch.autotune(ws, out, err, reps=2)
    _say("autotune", best.waves, best.chunk_groups, best.pairs_per_wave, ms)
    out.fill_(0x33)
    batch.decode(ws, out, err)
    torch.cuda.synchronize()
    assert int(err.item()) == 0
    _check_all(batch, out, mixed)


@pytest.mark.parametrize("shape", [(16, 4), (8, 4), (8, 8), (16, 8)])
@pytest.mark.parametrize("lanes,dt", [(32, np.uint8), (64, np.uint8), (32, np.uint16), (64, np.uint16)])
def test_single_stream_shapes(rc, shape, lanes, dt):
    A = 256 if dt == np.uint8 else 4096
    s = synth.draw_symbols(synth.zipf_pmf(A, 1.1), 5 + lanes, 150_001, dt)
    blob = rc.encode(s, lanes=lanes, quant_bits=12, splits=40, alphabet=A)
    plan = rc.Plan(blob)
    plan.set_tuning(waves=shape[0], chunk_groups=shape[1])
    ws = plan.allocate_workspace()
    plan.upload(ws)
    out = plan.allocate_output()
    out.fill_(0x77)
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    plan.decode(ws, out, err)
    torch.cuda.synchronize()
    assert int(err.item()) == 0
    assert np.array_equal(plan.symbols_of(out), s)


def _full_size_mix(rc, want_wide=3, want_narrow=5):
    """Streams of the mixed-batch configuration with sizes drawn from 8..16 MiB, of
    both table classes (uint8 / uint16 alphabets), about 8 KiB per split."""
    out, wide, narrow = [], 0, 0
    for i in range(64):
        spec = synth.mixed_stream_spec(3, i, 8 << 20, 16 << 20, 8 << 10)
        is_wide = spec.symbol_bytes == 2
        if (is_wide and wide >= want_wide) or (not is_wide and narrow >= want_narrow):
            continue
        s = spec.generate()
        present = int(np.count_nonzero(np.bincount(s, minlength=spec.alphabet)))
        n = max(spec.quant_bits, int(np.ceil(np.log2(max(present, 2)))))
        out.append((s, rc.encode(s, lanes=32, quant_bits=n, splits=spec.splits, alphabet=spec.alphabet)))
        wide += is_wide
        narrow += not is_wide
        if wide == want_wide and narrow == want_narrow:
            break
    assert wide == want_wide and narrow == want_narrow
    return out


def test_batch_full_size_streams(rc):
    """8..16 MiB streams of the mixed batch in both table classes, each spanning many
    work items: the autotuned graph replay and the per-stream baseline, every
    stream compared whole."""
    from paper_2306_12141_amd.batch import Batch
    streams = _full_size_mix(rc)
    batch = Batch([b for _, b in streams])
    ws, out, err = batch.allocate()
    batch.upload(ws)
    best, _ = batch.autotune(ws, out, err, reps=1)
    _say("full-size batch: items", batch.items, "tuning", best.waves, best.chunk_groups, best.pairs_per_wave,
         best.units_per_run, "splits", [b.splits for _, b in streams])
    assert batch.items > 2 * len(streams)
    g = batch.graph(ws, out, err)
    for rep in range(2):
        out.fill_(0x5A if rep else 0xA5)
        g.launch()
        torch.cuda.synchronize()
        assert int(err.item()) == 0
        _check_all(batch, out, streams)
    out.fill_(0x3C)
    batch.decode_per_stream(ws, out, err)
    torch.cuda.synchronize()
    assert int(err.item()) == 0
    _check_all(batch, out, streams)


def test_batch_with_partitioned_streams(rc, mixed):
    """Conventional partitioned streams (Sec. 2.3) batched with Recoil streams."""
    from paper_2306_12141_amd.batch import Batch
    extra = []
    for i, (W, N, P, dt) in enumerate([(32, 400_001, 300, np.uint8), (64, 200_000, 64, np.uint16),
                                       (32, 3_000, 7, np.uint8)]):
        A = 256 if dt == np.uint8 else 4096
        s = synth.draw_symbols(synth.zipf_pmf(A, 1.2), 1300 + i, N, dt)
        extra.append((s, rc.encode_partitioned(s, lanes=W, quant_bits=12, partitions=P, alphabet=A)))
    streams = mixed[:16] + extra
    batch = Batch([b for _, b in streams])
    ws, out, err = batch.allocate()
    batch.upload(ws)
    for rep in range(2):
        out.fill_(0x5A if rep else 0xA5)
        (batch.decode if rep == 0 else batch.decode_per_stream)(ws, out, err)
        torch.cuda.synchronize()
        assert int(err.item()) == 0
        _check_all(batch, out, streams)


def test_batch_offsets_past_2gib(rc, mixed):
    """A batch whose outputs end past 2^31 bytes: a 2 GiB + 77-symbol stream first,
    then the mixed streams, so their output offsets exceed 2^31."""
    from paper_2306_12141_amd.batch import Batch
    import synth
    N = (1 << 31) + 77
    big = synth.draw_symbols(synth.zipf_pmf(256, 1.1), 6300, N, np.uint8)
    _say("batch with a 2 GiB stream")
    streams = [(big, rc.encode(big, lanes=32, quant_bits=11, splits=32768))] + list(mixed[:8])
    batch = Batch([b for _, b in streams])
    ws, out, err = batch.allocate()
    batch.upload(ws)
    out.fill_(0xEE)
    batch.decode(ws, out, err)
    torch.cuda.synchronize()
    assert int(err.item()) == 0
    assert batch.output_range(len(streams) - 1)[0] > (1 << 31)
    _check_all(batch, out, streams)


def test_batch_with_wide_tables(rc, mixed):
    """Streams coded at 13 <= n <= 16 in a batch with one-level ones: three table
    classes, the wide one decoded by its own kernel; persistent, per-stream, graph
    replay and the allocation-free entry point all exact."""
    from paper_2306_12141_amd.batch import Batch
    import synth
    wide = []
    for i, (W, n, dt, A) in enumerate([(32, 16, np.uint8, 256), (64, 13, np.uint8, 256), (32, 15, np.uint16, 4096),
                                       (64, 16, np.uint16, 1000), (32, 16, np.uint8, 256)]):
        s = synth.draw_symbols(synth.zipf_pmf(A, 1.1), 6500 + i, 300_001 + 977 * i, dt)
        wide.append((s, rc.encode(s, lanes=W, quant_bits=n, splits=40 + i, alphabet=A)))
    streams = list(mixed[:12]) + wide
    _say("batch with wide tables", len(streams))
    batch = Batch([b for _, b in streams])
    ws, out, err = batch.allocate()
    batch.upload(ws)
    for run in ("persistent", "per_stream", "graph", "noalloc"):
        out.fill_(0x3C)
        if run == "persistent":
            batch.decode(ws, out, err)
        elif run == "per_stream":
            batch.decode_per_stream(ws, out, err)
        elif run == "graph":
            g = batch.graph(ws, out, err)
            g.launch()
        else:
            batch.decode_noalloc(ws, out, err)
        torch.cuda.synchronize()
        assert int(err.item()) == 0, run
        _check_all(batch, out, streams)
