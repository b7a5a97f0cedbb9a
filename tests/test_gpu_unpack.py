"""GPU parity of the device-side metadata unpacker (packed plans).

A packed plan uploads the container's packed metadata section and a kernel
writes the per-unit and per-lane records into the workspace. They must equal,
word for word, the records the host planner uploads for the same stream
combined to the same number of units (whose reading of the section is checked
on the CPU in tests/test_packed_plan.py); the workspace is filled with a
pattern first, so a record left unwritten is caught. The decode that follows
must reproduce the input symbols exactly.
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


def _syms(seed, n, A, dtype=np.uint8, skew=None):
    if skew is None:
        return (synth.splitmix64(seed, 0, n) % np.uint64(A)).astype(dtype)
    return synth.draw_symbols(synth.zipf_pmf(A, skew), seed, n, dtype)


def _uploaded(plan, fill):
    ws = plan.allocate_workspace()
    ws.fill_(fill)
    plan.upload(ws)
    torch.cuda.synchronize()
    return ws


def _decode(plan, ws, table_index=None):
    out = plan.allocate_output()
    out.fill_(0xA5)
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    if table_index is None:
        plan.decode(ws, out, err)
    else:
        plan.decode_adaptive(ws, table_index, out, err)
    torch.cuda.synchronize()
    assert int(err.item()) == 0
    return plan.symbols_of(out)


def _check(rc, blob, s, targets, table_index=None):
    M = blob.splits
    for t in targets:
        _say("  target", t)
        packed = rc.Plan(blob, packed_target=t)
        host = rc.Plan(blob.combine(t) if 0 < t < M else blob)
        ws_p = _uploaded(packed, 0xC3)
        ws_h = _uploaded(host, 0x3C)
        rp, lp = packed.device_records(ws_p)
        rh, lh = host.device_records(ws_h)
        assert np.array_equal(rp, host.units()), f"target {t}: unit records"
        assert np.array_equal(rp, rh) and np.array_equal(lp, lh), f"target {t}: lane words"
        assert np.array_equal(_decode(packed, ws_p, table_index), s), f"target {t}: symbols"
        # The unpack alone (recoil_plan_unpack) rewrites records that were overwritten.
        lay = packed.layout()
        ws_p[lay.units: lay.total if lay.unit_count == 0 else lay.lanes + 4 * lay.unit_count * lay.lanes_per_unit] \
            .fill_(0xEE)
        packed.unpack(ws_p)
        torch.cuda.synchronize()
        rp2, lp2 = packed.device_records(ws_p)
        assert np.array_equal(rp2, rp) and np.array_equal(lp2, lp), f"target {t}: unpack again"


CASES = [
    # lanes, n, dtype, alphabet, N, splits, zipf
    (32, 11, np.uint8, 256, 1 << 20, 256, 1.1),
    (64, 11, np.uint8, 256, 1 << 20, 300, 0.9),
    (32, 12, np.uint16, 4096, 300_003, 64, 1.2),
    (64, 12, np.uint16, 4096, 120_003, 20, 1.3),
    (32, 8, np.uint8, 3, 40_000, 30, 2.5),
    (64, 11, np.uint8, 256, 65, 4, None),
    (32, 11, np.uint8, 256, 31, 4, None),
    (32, 11, np.uint8, 256, 1, 1, None),
]


@pytest.mark.parametrize("ci", range(len(CASES)), ids=[f"W{c[0]}_{np.dtype(c[2]).name}_N{c[4]}_M{c[5]}" for c in CASES])
def test_unpack_matches_host(rc, ci):
    W, n, dt, A, N, M, z = CASES[ci]
    _say("case", CASES[ci])
    s = _syms(5000 + ci, N, A, dt, z)
    blob = rc.encode(s, lanes=W, quant_bits=n, splits=M, alphabet=A)
    _check(rc, blob, s, sorted({0, 1, 2, 3, max(1, M // 3), max(1, M - 1), M, M + 5}))


def test_unpack_full_stream_every_target_shape(rc):
    """A 64 MiB stream with 2048 units, unpacked whole and combined."""
    N = 1 << 26
    s = _syms(5100, N, 256, np.uint8, 1.1)
    _say("case full W=32 N=2^26 M=2048")
    blob = rc.encode(s, lanes=32, quant_bits=11, splits=2048)
    _check(rc, blob, s, [0, 1000, 77])


def test_unpack_adaptive(rc, orc):
    T, A, nbits, M, N = 16, 64, 9, 512, 2_000_003
    pmfs, tidx, s = synth.adaptive_stream(5200, N, T, A)
    tabs = np.stack([orc.quantize((pmf * (1 << 30)).astype(np.uint64) + 1, nbits) for pmf in pmfs])
    _say("case adaptive", T, A, nbits, M, N)
    blob = rc.encode_adaptive(s, tabs, tidx, lanes=32, quant_bits=nbits, splits=M, alphabet=A)
    _check(rc, blob, s, [0, 100], table_index=torch.from_numpy(tidx).to("cuda"))


def test_unpack_reupload_smaller(rc):
    """One workspace, two packed plans in a row (the second with fewer units):
    the second upload's records replace the first's."""
    s = _syms(5300, 1 << 20, 256, np.uint8, 1.0)
    blob = rc.encode(s, lanes=64, quant_bits=11, splits=400)
    big, small = rc.Plan(blob, packed_target=0), rc.Plan(blob, packed_target=9)
    ws = big.allocate_workspace()
    ws.fill_(0x77)
    big.upload(ws)
    assert np.array_equal(_decode(big, ws), s)
    assert small.device_bytes <= big.device_bytes
    small.upload(ws[: small.device_bytes])
    torch.cuda.synchronize()
    rec, _ = small.device_records(ws[: small.device_bytes])
    assert np.array_equal(rec, rc.Plan(blob.combine(9)).units())
    assert np.array_equal(_decode(small, ws[: small.device_bytes]), s)
