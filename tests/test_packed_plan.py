"""Packed plans (the split metadata unpacked on the device): host-side checks.

The unpacker's reading of the packed metadata section (Sec. 4.3: offset and
group series, then per split point the lane states and a group-difference
series) is restated in tests/_fmt.py and checked here against the host
planner's records of the combined stream and against the oracle encoder's own
split records (lane states and symbol indices). The device kernel is checked
against the host planner in tests/test_gpu_unpack.py. Runs on the CPU.
"""

import numpy as np
import pytest

import synth
from tests._fmt import parse, unit_records


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
    (32, 11, np.uint8, 256, 300_001, 64, 1.1),
    (64, 12, np.uint8, 256, 200_000, 37, 0.9),
    (32, 12, np.uint16, 4096, 120_003, 20, 1.2),
    (32, 8, np.uint8, 3, 40_000, 30, 2.5),
    (64, 11, np.uint8, 256, 65, 4, None),
    (32, 11, np.uint8, 256, 1, 1, None),
]
TARGETS = [0, 1, 2, 3, 7, 1000]


@pytest.mark.parametrize("ci", range(len(CASES)))
def test_reading_matches_host_planner(rc, ci):
    """Records read from the packed section equal the host planner's records of
    the combined stream, for every target."""
    W, n, dt, A, N, M, z = CASES[ci]
    s = _syms(4000 + ci, N, A, dt, z)
    blob = rc.encode(s, lanes=W, quant_bits=n, splits=M, alphabet=A)
    c = blob.to_bytes()
    for t in TARGETS + [M - 1, M]:
        rec, _ = unit_records(c, t)
        host = rc.Plan(blob.combine(t) if 0 < t < blob.splits else blob).units()
        assert np.array_equal(rec, host), f"target {t}"


def test_lane_words_match_oracle_splits(rc, orc):
    """Lane words: the oracle encoder's recorded state of each lane at the split
    point, and the lane's activation step = anchor group - its symbol's group."""
    W, N, M = 32, 200_003, 40
    s = _syms(4100, N, 256, np.uint8, 1.0)
    p = orc.params(lanes=W, quant_bits=11, alphabet=256)
    enc = orc.encode(s, p, M)
    c = enc.container()
    rec, lanes = unit_records(c, 0)
    for k in range(1, M):
        sp = enc.split(k)
        top = sp.imax // W
        assert rec[k - 1][1] == top
        assert np.array_equal(lanes[k - 1] & 0xFFFF, sp.states & 0xFFFF)
        assert np.array_equal(lanes[k - 1] >> 16, top - sp.indices // W)
    assert np.array_equal(lanes[M - 1], parse(c)["final"])


def test_packed_plan_layout(rc):
    W, N, M = 64, 500_000, 300
    s = _syms(4200, N, 256, np.uint8, 1.2)
    blob = rc.encode(s, lanes=W, quant_bits=11, splits=M)
    meta_bytes = len(parse(blob.to_bytes())["meta"])
    for t, units in [(0, M), (M, M), (M + 9, M), (150, 150), (7, 7), (1, 1), (299, 150), (100, 100), (101, 100)]:
        plan = rc.Plan(blob, packed_target=t)
        lay = plan.layout()
        assert lay.packed == 1 and lay.lanes_per_unit == W
        assert lay.unit_count == units, t
        assert lay.total == plan.device_bytes
        assert plan.metadata_device_bytes == meta_bytes + 4 * (M - 1) + 4 * W
        with pytest.raises(rc.RecoilError, match="unsupported"):
            plan.units()
    host = rc.Plan(blob)
    assert host.layout().packed == 0 and host.layout().unit_count == M
    assert host.metadata_device_bytes == 16 * M + 4 * W * M


def test_packed_plan_rejects(rc, orc):
    s = _syms(4300, 100_000, 256, np.uint8, 1.0)
    part = rc.encode_partitioned(s, lanes=32, quant_bits=11, partitions=16)
    with pytest.raises(rc.RecoilError, match="unsupported"):
        rc.Plan(part, packed_target=0)
    narrow = rc.encode(s, lanes=16, quant_bits=11, splits=8)
    with pytest.raises(rc.RecoilError, match="unsupported"):
        rc.Plan(narrow, packed_target=0)
