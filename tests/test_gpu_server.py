"""GPU tests of the serving loop: every request decodes to its content's symbols,
alone and mixed with others, under budget pressure, and oversize requests are
refused without blocking the queue.

Expected outputs are the seeded input symbols (lossless codec); comparisons are
bit-exact.
"""

import sys
import time

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


@pytest.fixture(scope="module")
def corpus(rc):
    """Twelve streams of the serving mix (16 KiB .. 1 MiB, about 1 KiB per split)."""
    out = []
    for i in range(12):
        spec = synth.mixed_stream_spec(41, i, 16 << 10, 1 << 20, 1 << 10)
        s = spec.generate()
        present = int(np.count_nonzero(np.bincount(s, minlength=spec.alphabet)))
        n = max(spec.quant_bits, int(np.ceil(np.log2(max(present, 2)))))
        if i == 5:
            s = np.full(3000, 9, dtype=spec.dtype)      # single-symbol content
        blob = rc.encode(s, lanes=64 if i % 4 == 3 else 32, quant_bits=n, splits=spec.splits,
                         alphabet=spec.alphabet)
        out.append((s, blob))
    return out


def _combined_units(m, target):
    """Units left after keeping every ceil(m / target)-th split point."""
    step = -(-m // min(target, m))
    return (m - 1) // step + 1


def _align(v):
    return (v + 255) // 256 * 256


def _server(rc, corpus, budget_bytes, hip_streams=2, max_batch=256, items_per_launch=4096):
    """A server whose request budget is exactly budget_bytes (arena = resident
    region + one control region per stream + budget)."""
    from paper_2306_12141_amd.server import Server
    resident = _align(sum(b.info.n_words * 2 + (64 << 10) for _, b in corpus))
    # Control region per stream: queue head, error words, item counts, descriptors, items.
    ctrl = _align(256 + 2 * _align(max_batch * 4) + _align(max_batch * 64) + items_per_launch * 16)
    arena = torch.empty(resident + hip_streams * ctrl + _align(budget_bytes), dtype=torch.uint8, device="cuda")
    srv = Server(arena, resident, hip_streams=hip_streams, max_batch=max_batch,
                 items_per_launch=items_per_launch)
    assert srv.stats().budget_bytes == _align(budget_bytes)
    ids = [srv.add_content(b) for _, b in corpus]
    return srv, ids


def _drain(srv, want, timeout_s=60.0):
    got = {}
    t0 = time.time()
    while len(got) < want:
        for c in srv.poll(timeout_us=2000):
            got[c.request_id] = c
        assert time.time() - t0 < timeout_s, f"only {len(got)} of {want} completions"
    return got


def _check(srv, corpus, c):
    s, _ = corpus[c.content]
    assert c.status == 0, f"request {c.request_id}: status {c.status}"
    assert c.device_error == 0
    assert c.out_bytes == s.nbytes
    got = srv.output_of(c, s.dtype)
    assert np.array_equal(got, s), f"request {c.request_id} content {c.content} splits {c.splits}"
    assert c.t_arrival_ns <= c.t_admit_ns <= c.t_launch_ns <= c.t_done_ns


def test_alone(rc, corpus):
    srv, ids = _server(rc, corpus, 64 << 20)
    try:
        for cid in ids:
            for splits in (1, 7, 0):
                rid = srv.submit(cid, splits, tag=cid)
                got = _drain(srv, 1)
                c = got[rid]
                _check(srv, corpus, c)
                blob = corpus[cid][1]
                full = blob.splits
                assert c.splits == (full if splits == 0 else _combined_units(full, splits))
                # The size a client would receive equals the combined container's metadata section.
                ref = blob if splits == 0 else blob.combine(splits)
                assert c.metadata_bytes == ref.info.metadata_bytes
                srv.release(rid)
        st = srv.stats()
        assert st.completed == 3 * len(ids) and st.budget_used == 0 and st.pending == 0
    finally:
        srv.close()


def test_mixed_continuous_batching(rc, corpus):
    """Many requests in flight at once: each output equals the one it has alone."""
    srv, ids = _server(rc, corpus, 256 << 20, hip_streams=3, max_batch=16)
    try:
        reqs = {}
        for k in range(96):
            cid = ids[(k * 7) % len(ids)]
            full = corpus[cid][1].splits
            splits = synth.log_uniform_int(91, k, 1, full)
            reqs[srv.submit(cid, splits, tag=k)] = cid
        got = _drain(srv, len(reqs))
        for rid, c in got.items():
            assert c.content == reqs[rid]
            _check(srv, corpus, c)
            srv.release(rid)
        st = srv.stats()
        _say("launches", st.launches, "requests", st.requests_launched, "peak budget", st.budget_peak)
        assert st.launches < len(reqs)          # requests were folded into shared launches
        assert st.budget_used == 0
    finally:
        srv.close()


def test_budget_pressure_and_oversize(rc, corpus):
    """A budget that holds the largest output and little more: requests wait for
    releases and still decode exactly; one larger than the whole budget is
    refused and does not block the queue."""
    big = max(range(len(corpus)), key=lambda i: corpus[i][0].nbytes)
    biggest = corpus[big][0].nbytes
    total = sum(corpus[(k * 5 + big) % len(corpus)][0].nbytes for k in range(30))
    assert total > 4 * (biggest + (1 << 20))
    srv, ids = _server(rc, corpus, biggest + (1 << 20), hip_streams=2, max_batch=4)
    try:
        pending = {}
        for k in range(30):
            cid = ids[(k * 5 + big) % len(ids)]
            pending[srv.submit(cid, 0, tag=k)] = cid
        done = 0
        t0 = time.time()
        while done < len(pending):
            for c in srv.poll(timeout_us=2000):
                _check(srv, corpus, c)
                srv.release(c.request_id)
                done += 1
            assert time.time() - t0 < 60
        st = srv.stats()
        assert st.budget_peak <= st.budget_bytes and st.budget_used == 0
    finally:
        srv.close()
    # A budget smaller than one output: the request is refused, later ones run.
    small = min(range(len(corpus)), key=lambda i: corpus[i][0].nbytes)
    budget = _align(corpus[small][0].nbytes) + (256 << 10)
    assert corpus[big][0].nbytes > budget
    srv, ids = _server(rc, corpus, budget)
    try:
        r_big = srv.submit(ids[big], 0)
        r_small = srv.submit(ids[small], 0)
        got = _drain(srv, 2)
        assert got[r_big].status == -5          # RECOIL_ERR_BUFFER_TOO_SMALL
        _check(srv, corpus, got[r_small])
    finally:
        srv.close()


@pytest.fixture(scope="module")
def big_corpus(rc):
    """Two serving contents of at least 16 MiB (uint8 and uint16, W = 32), stored with
    about 1 KiB per split."""
    out = []
    for i, (wide, mib) in enumerate([(False, 20), (True, 16)]):
        A, dt = (4096, np.uint16) if wide else (256, np.uint8)
        n_sym = (mib << 20) // (2 if wide else 1)
        s = synth.draw_symbols(synth.laplace_pmf(A, A / 2, 6.0 + 10 * i), 4200 + i, n_sym, dt)
        present = int(np.count_nonzero(np.bincount(s, minlength=A)))
        n = max(11, int(np.ceil(np.log2(max(present, 2)))))
        blob = rc.encode(s, lanes=32, quant_bits=n, splits=-(-s.nbytes // 1024), alphabet=A)
        out.append((s, blob))
    return out


def test_full_size_requests(rc, big_corpus):
    """Requests for 16..20 MiB contents combined to one unit, a few units and all units:
    each alone, then all of them in flight together; every output compared whole."""
    srv, ids = _server(rc, big_corpus, 512 << 20, hip_streams=3, max_batch=16, items_per_launch=1 << 16)
    try:
        asks = [(cid, k) for cid in ids for k in (1, 3, 0)]
        for cid, k in asks:
            rid = srv.submit(cid, k, tag=cid)
            c = _drain(srv, 1, timeout_s=120)[rid]
            full = big_corpus[cid][1].splits
            assert c.splits == (full if k == 0 else _combined_units(full, k))
            _check(srv, big_corpus, c)
            srv.release(rid)
        reqs = {srv.submit(cid, k, tag=j): (cid, k) for j, (cid, k) in enumerate(asks + asks)}
        got = _drain(srv, len(reqs), timeout_s=120)
        for rid, c in got.items():
            assert c.content == reqs[rid][0]
            _check(srv, big_corpus, c)
            srv.release(rid)
        assert srv.stats().budget_used == 0
    finally:
        srv.close()


def test_add_content_refuses_streams_decoded_alone(rc, corpus):
    """Conventional partitioned and adaptive streams are refused at add_content with
    RECOIL_ERR_UNSUPPORTED; the server keeps serving."""
    srv, ids = _server(rc, corpus, 16 << 20)
    try:
        s = synth.draw_symbols(synth.zipf_pmf(256, 1.1), 6400, 100_000, np.uint8)
        pmfs, tidx, sa = synth.adaptive_stream(6401, 100_000, 4, 64)
        tabs = np.stack([rc.quantize((pmf * (1 << 30)).astype(np.uint64) + 1, 10) for pmf in pmfs])
        refused = [rc.encode_partitioned(s, lanes=32, quant_bits=11, partitions=8),
                   rc.encode_adaptive(sa, tabs, tidx, lanes=32, quant_bits=10, splits=16, alphabet=64)]
        for b in refused:
            with pytest.raises(rc.RecoilError) as e:
                srv.add_content(b)
            assert e.value.status == -4
        rid = srv.submit(ids[0], 3, tag=0)
        _check(srv, corpus, _drain(srv, 1)[rid])
        srv.release(rid)
    finally:
        srv.close()


def test_wide_table_content(rc, corpus):
    """Content coded at 13 <= n <= 16 served beside one-level content: each launch
    runs the wide requests' items in a second persistent kernel."""
    wide = []
    for i, (W, n, dt, A) in enumerate([(32, 16, np.uint8, 256), (64, 14, np.uint8, 256), (32, 16, np.uint16, 2000)]):
        s = synth.draw_symbols(synth.zipf_pmf(A, 1.2), 6600 + i, 200_003 + 311 * i, dt)
        wide.append((s, rc.encode(s, lanes=W, quant_bits=n, splits=64, alphabet=A)))
    allc = list(corpus) + wide
    srv, ids = _server(rc, allc, 64 << 20)
    try:
        rids = []
        for rep in range(3):
            for cid in ids:
                rids.append(srv.submit(cid, (3, 0, 17)[rep], tag=cid))
        got = _drain(srv, len(rids))
        for rid in rids:
            _check(srv, allc, got[rid])
            srv.release(rid)
    finally:
        srv.close()
