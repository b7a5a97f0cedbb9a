"""recoil_decode_batch_noalloc (queue heads in the library's static device
array) against recoil_decode_batch (heads in the workspace), through the C ABI.

Two calls in a row on one GPU, the second on a smaller batch, so the second
call finds the heads the first one left behind. Each output is compared byte
for byte with the existing entry point's output and with the seeded input
symbols; the workspace must come out of the no-allocation call unchanged.
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


def _streams(rc, count, seed):
    """Mixed streams of both table classes (uint8 and uint16), W 32 and 64."""
    out = []
    for i in range(count):
        spec = synth.mixed_stream_spec(seed, i, 1 << 12, 1 << 20, 4 << 10)
        s = spec.generate()
        present = int(np.count_nonzero(np.bincount(s, minlength=spec.alphabet)))
        n = max(spec.quant_bits, int(np.ceil(np.log2(max(present, 2)))))
        lanes = 64 if i % 4 == 3 else 32
        out.append((s, rc.encode(s, lanes=lanes, quant_bits=n, splits=spec.splits, alphabet=spec.alphabet)))
    return out


def _ranges_equal(batch, a, b, streams):
    for i, (s, _) in enumerate(streams):
        off, n = batch.output_range(i)
        assert torch.equal(a[off:off + n], b[off:off + n]), f"stream {i}: outputs of the two entry points differ"
        got = a[off:off + n].cpu().numpy().view(s.dtype)
        assert np.array_equal(got, s), f"stream {i}: output differs from the input symbols"


@pytest.mark.parametrize("call,count,seed", [(1, 40, 801), (2, 9, 802)])
def test_noalloc_matches_decode_batch(rc, call, count, seed):
    from paper_2306_12141_amd.batch import Batch
    streams = _streams(rc, count, seed)
    assert {s.dtype for s, _ in streams} == {np.dtype(np.uint8), np.dtype(np.uint16)}
    batch = Batch([b for _, b in streams])
    _say(f"call {call}: {count} streams, {batch.items} items")
    ws, ref, err_ref = batch.allocate()
    batch.upload(ws)
    ref.fill_(0x3C)
    batch.decode(ws, ref, err_ref)
    torch.cuda.synchronize()
    assert int(err_ref.item()) == 0
    ws_before = ws.clone()
    out = torch.full_like(ref, 0xC3)
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    batch.decode_noalloc(ws, out, err)
    torch.cuda.synchronize()
    assert int(err.item()) == 0
    assert torch.equal(ws, ws_before), "the no-allocation decode wrote to the workspace"
    _ranges_equal(batch, out, ref, streams)
