#!/usr/bin/env python3
"""Recoil decode benchmark on one MI355X.

Headline (`value`): a single 256 MiB uint8 stream, iid Zipf(s = 1.1) over a
seeded permutation of 256 symbols, n = 12, W = 64 interleaved lanes (--lanes),
encoded with 65536 splits. One step is one recoil_decode of the whole stream
with the bitstream, table and metadata already resident in HBM. `value` is
decoded output bytes per second (1 GB = 1e9 B) over the timed steps.

The same line also carries (each bit-exact against the input symbols):
  extras: the stream at W = 32, every split point used, a decode after evicting
      the caches, the W = 32 stream combined to 16384 / 4096 / 1024 / 256 splits,
      the same stream coded by the conventional partitioning baseline (Sec. 2.3) at
      65536 / 16384 / 2176 / 256 / 16 sub-sequences against Recoil at the same
      parallelism (2176 and 16: the paper's Large and Small variations),
      adaptive coding (16 per-symbol tables) against one static table on the same
      symbols, the headline stream coded at n = 16 (two-level table), the split
      metadata unpacked on the device against the host planner, the host encode
      with the streaming and the threaded split writer, the small Laplace stream,
      and the host-to-device upload;
  c3: 4096 mixed streams (4 KiB..16 MiB, Laplace/Zipf/uniform, uint8 and uint16,
      n 10..12, about 8 KiB per split) decoded by one hipGraph replay of the
      persistent batched kernel (autotuned launch shape) versus one single-stream
      launch per stream, every stream of both checked;
  c4: the serving loop, Poisson arrivals at 2000 requests/s over a resident corpus
      of 64 KiB..64 MiB streams stored with about 1 KiB per split; each request
      asks for a log-uniform number of decode units (combined at admission);
      32 GiB request budget; sustained decoded GB/s and p50/p99/p99.9 latency
      from arrival to observed completion, every request's output compared on
      the device with its content before release.
Each carries `roofline` (HBM and ALU ceilings of its dominant kernel) and
`cpu_baseline` (the CPU oracle on a bounded sample of the same workload).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload all|c1|c3|c4|n16]
Prints exactly one JSON line on stdout; progress goes to stderr.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Plain-ALU peak: 256 CUs x 4 SIMDs at the 2.4 GHz peak engine clock. A SIMD
# executes a wave64 VALU instruction in 4 cycles (16 lanes per cycle) and can issue
# two in the same 4 cycles (SQ_ACTIVE_INST_VALU2 counts such quad-cycles), so its
# peak is 32 lane-operations per cycle: the rate behind the published fp32 vector
# peak (1024 x 32 lanes x 2 flops per FMA x 2.4 GHz = 157.3 TFLOP/s).
SIMDS = 256 * 4
CLOCK_GHZ = 2.4
VALU_LANES_PER_CYCLE = 32
VALU_PEAK_TLANEOPS = SIMDS * VALU_LANES_PER_CYCLE * CLOCK_GHZ / 1e3      # 78.64 T int32 lane-ops/s
METRIC = "decoded GB/s on 1 MI355X (batched vs per-stream launch, bit-exact); p99 latency"

DEV = "paper_2306_12141_amd/csrc/device/"
KERNEL_SOURCES = {
    "decode_units": (DEV + "decode.hip", DEV + "decode.hpp", DEV + "decode_core.hpp"),
    "decode_batch": (DEV + "batch.hip", DEV + "batch.hpp", DEV + "decode.hpp", DEV + "decode_core.hpp"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash(kernel: str = "decode_units") -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _profile_record(fname: str, key: str, kernel: str):
    """A committed per-launch record from rocprofv3 counter runs, if it was taken on this kernel source."""
    try:
        with open(os.path.join(ROOT, "profiles", fname)) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    ent = rec.get(key)
    if not ent or ent.get("kernel_hash") != kernel_source_hash(kernel):
        return None
    return ent


def measured_traffic(key: str, kernel: str = "decode_units"):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None."""
    ent = _profile_record("traffic.json", key, kernel)
    return ent.get("bytes_per_launch") if ent else None


def roofline(key: str, kernel: str, alg_bytes: int, kernel_ms: float, **extra) -> dict:
    """Position of one kernel against both ceilings that can bind it.

    HBM: algorithmic bytes per launch / mean launch duration against 8 TB/s.
    ALU: the VALU instructions one launch issues (SQ_INSTS_VALU, from committed
    counter runs of this kernel source) need count x 2 cycles / (1024 SIMDs x
    2.4 GHz) at the least (two wave64 instructions per SIMD every 4 cycles); as a
    rate, count x 64 lanes / duration against 78.6 T int32 lane-ops/s. `bound` is
    the ceiling with the longer floor; the top-level achieved/peak/frac are that
    ceiling's."""
    hbm_gbs = alg_bytes / (kernel_ms * 1e-3) / 1e9
    hbm = {"achieved": round(hbm_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(hbm_gbs / HBM_PEAK_GBS, 4),
           "ceiling_ms": round(alg_bytes / (HBM_PEAK_GBS * 1e9) * 1e3, 5)}
    cnt = _profile_record("counters.json", key, kernel)
    alu = None
    if cnt and cnt.get("per_launch", {}).get("SQ_INSTS_VALU"):
        valu = float(cnt["per_launch"]["SQ_INSTS_VALU"])
        lane_ops = valu * 64
        ach = lane_ops / (kernel_ms * 1e-3) / 1e12
        alu = {"achieved": round(ach, 2), "peak": round(VALU_PEAK_TLANEOPS, 2), "unit": "T int32 lane-ops/s",
               "frac": round(ach / VALU_PEAK_TLANEOPS, 4),
               "ceiling_ms": round(valu * 64 / VALU_LANES_PER_CYCLE / (SIMDS * CLOCK_GHZ * 1e9) * 1e3, 5),
               "valu_per_launch": int(valu), "salu_per_launch": cnt["per_launch"].get("SQ_INSTS_SALU"),
               "dual_issue_quad_cycles": cnt["per_launch"].get("SQ_ACTIVE_INST_VALU2"),
               "valu_per_64_symbols": cnt.get("valu_per_64_symbols"),
               "source": f"profiles/counters.json[{key}]"}
    top = alu if alu and alu["ceiling_ms"] > hbm["ceiling_ms"] else hbm
    out = {"bound": "alu" if top is alu else "hbm", "achieved": top["achieved"], "peak": top["peak"],
           "unit": top["unit"], "frac": top["frac"], "traffic": measured_traffic(key, kernel), "kernel": kernel,
           "alg_bytes_per_launch": alg_bytes, "kernel_ms_mean": round(kernel_ms, 5), "hbm": hbm, "alu": alu}
    out.update(extra)
    if alu is None and not cnt:
        out["alu_note"] = f"no committed counter run of this kernel source for {key}"
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_cores() -> int:
    """Host threads the CPU legs use: the CPUs this process may run on, at most 16
    (one GPU's share of the host on the benchmark machines)."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return max(1, min(n, 16))


# Untimed decoding before the warm-up steps, in milliseconds. An idle MI355X sits at a
# deep-sleep clock and needs some tens of milliseconds of load to reach its steady clock
# (from 157 MHz: the first 25 decodes averaged 203 us, decodes 200 on 120 us, at 2.28 GHz
# and about 1.2 kW); without it the timed steps would measure the ramp.
SETTLE_MS = 40.0


def settle(fn, torch, ms=SETTLE_MS):
    """Run fn back to back until `ms` of wall time have passed; returns the launches made."""
    n = 0
    t0 = time.perf_counter()
    while (time.perf_counter() - t0) * 1e3 < ms:
        for _ in range(8):
            fn()
        n += 8
        torch.cuda.synchronize()
    return n


def time_decode(plan, ws, out, err, steps, warmup, torch):
    """Timed region: `steps` decodes launched back to back on the current stream between
    two HIP events, after the clock-settling decodes and `warmup` untimed ones. Their mean
    launch duration (total / steps, inter-launch gaps included) is the kernel time the
    roofline uses. A second, untimed pass puts an event pair around every launch for the
    spread of single launches; those events add a gap of several microseconds between
    launches, which is why they stay out of the timed region."""
    settled = settle(lambda: plan.decode(ws, out, err), torch)
    for _ in range(warmup):
        plan.decode(ws, out, err)
    torch.cuda.synchronize()
    t_all0 = torch.cuda.Event(enable_timing=True)
    t_all1 = torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    t_all0.record()
    for _ in range(steps):
        plan.decode(ws, out, err)
    t_all1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = t_all0.elapsed_time(t_all1)
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    for k in range(steps):
        starts[k].record()
        plan.decode(ws, out, err)
        ends[k].record()
    torch.cuda.synchronize()
    per = sorted(s.elapsed_time(e) for s, e in zip(starts, ends))
    return {"ms_total": total_ms, "ms_per_step": total_ms / steps, "kernel_ms_mean": total_ms / steps,
            "kernel_ms_median": per[len(per) // 2], "kernel_ms_min": per[0], "wall_s": wall,
            "settle_launches": settled}


def time_cold(plan, ws, out, err, torch, reps=9, evict_bytes=1 << 30):
    """Single decodes, each right after reading `evict_bytes` of other device memory
    (evicts the last-level cache without leaving dirty lines): how much the timed
    back-to-back decodes gain from the cache keeping part of the stream."""
    junk = torch.ones(evict_bytes // 8, dtype=torch.int64, device="cuda")
    per = []
    for _ in range(reps):
        junk.sum()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        plan.decode(ws, out, err)
        b.record()
        torch.cuda.synchronize()
        per.append(a.elapsed_time(b))
    del junk
    per.sort()
    return {"median_ms": round(per[len(per) // 2], 5), "min_ms": round(per[0], 5), "evicted_bytes": evict_bytes,
            "how": "one decode after reading the evicted bytes, HIP events around the decode"}


def check_exact(plan, out, symbols, err, np):
    got = plan.symbols_of(out)
    ok = bool(np.array_equal(got, symbols)) and int(err.item()) == 0
    return ok


def _median_time(fn, reps: int = 3):
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
    return sorted(ts)[len(ts) // 2]


def cpu_oracle_baseline(spec, sample_symbols: int, np):
    """The oracle, as it stands, on a bounded prefix of the same stream: (i) serial
    whole-stream interleaved decode on 1 core, (ii) per-split decode of every unit on 1
    core (synchronisation included), (iii) the same over all host threads. Median of 3
    runs each; `value` is (iii)."""
    import oracle
    import synth
    sub = synth.StreamSpec(**{**spec.__dict__, "n_symbols": min(sample_symbols, spec.n_symbols)})
    s = sub.generate()
    splits = max(1, int(spec.splits * len(s) / spec.n_symbols))
    p = oracle.params(lanes=spec.lanes, quant_bits=spec.quant_bits, symbol_bytes=spec.symbol_bytes,
                      alphabet=spec.alphabet)
    dec = oracle.Decoder(oracle.encode(s, p, splits).container())
    cores = host_cores()
    nbytes = len(s) * spec.symbol_bytes
    assert np.array_equal(dec.serial(), s) and np.array_equal(dec.all(aligned=True, workers=cores), s)
    t_serial = _median_time(lambda: dec.serial())
    t_one = _median_time(lambda: dec.all(aligned=True, workers=1))
    t_all = _median_time(lambda: dec.all(aligned=True, workers=cores))
    gbs = lambda t: round(nbytes / t / 1e9, 4)
    return {"value": gbs(t_all), "unit": "GB/s", "cores": cores, "kind": "oracle",
            "cpu": cpu_model(),
            "timings": {"serial_whole_stream_1_core": gbs(t_serial), "per_split_1_core": gbs(t_one),
                        f"per_split_{cores}_threads": gbs(t_all)},
            "sample": f"first {len(s)} symbols of the workload ({nbytes / 2**20:.0f} MiB), encoded by the oracle "
                      f"with {splits} splits (same symbols per split); value = all {splits} decode units over "
                      f"{cores} std::threads, {t_all:.3f} s (median of 3); 1 core: serial {t_serial:.2f} s, "
                      f"per-split {t_one:.2f} s"}


def cpu_oracle_streams(containers, np, symbols, label: str, budget_s: float = 12.0):
    """The oracle decoding whole containers one after another, each with all its units
    spread over the host threads (a unit per thread at a time), until about budget_s
    of wall time; every output checked."""
    import oracle
    cores = host_cores()
    done, nbytes, t = 0, 0, 0.0
    for c, s in zip(containers, symbols):
        dec = oracle.Decoder(c)
        t0 = time.perf_counter()
        out = dec.all(aligned=True, workers=min(cores, dec.threads))
        t += time.perf_counter() - t0
        assert np.array_equal(out, s), f"{label}: oracle output differs"
        done += 1
        nbytes += s.nbytes
        if t > budget_s:
            break
    return {"value": round(nbytes / t / 1e9, 4), "unit": "GB/s", "cores": cores, "kind": "oracle",
            "cpu": cpu_model(),
            "sample": f"{label}: {done} streams, {nbytes / 2**20:.0f} MiB decoded, each by the oracle's per-split "
                      f"decoder over min({cores}, its units) std::threads, {t:.2f} s"}


def algorithmic_bytes(spec, info, runs):
    """Bytes a decode must move: the symbols written, the bitstream read, per run
    the top unit's record (16 B), the bottom unit's last group (4 B) and the top
    unit's lane records (4 W B), and the decode table (2^n x 4 B)."""
    return (spec.n_symbols * spec.symbol_bytes + 2 * info.n_words + runs * (20 + 4 * info.lanes)
            + (4 << spec.quant_bits))


def run_c1(args, torch, np, rc, synth):
    lanes = args.lanes
    spec = synth.c1_spec(lanes)
    t0 = time.perf_counter()
    s = spec.generate()
    log(f"generated {spec.n_symbols} symbols in {time.perf_counter() - t0:.1f}s")
    t0 = time.perf_counter()
    blob = rc.encode(s, lanes=lanes, quant_bits=spec.quant_bits, splits=spec.splits)
    info = blob.info
    log(f"encoded: {info.n_words} words, {info.splits} splits, metadata {info.metadata_bytes} B "
        f"in {time.perf_counter() - t0:.1f}s")
    plan = rc.Plan(blob)
    if args.shape:
        v = [int(x) for x in args.shape.split(",")]
        plan.set_tuning(waves=v[0], chunk_groups=v[1], blocks_per_cu=v[2], units_per_run=v[3] if len(v) > 3 else 0)
    shape = plan.shape()
    ws = plan.allocate_workspace()
    # First upload (includes one-time driver and staging set-up), then a warm one.
    upload = []
    for _ in range(2):
        torch.cuda.synchronize()
        t_up = time.perf_counter()
        plan.upload(ws)
        torch.cuda.synchronize()
        upload.append(time.perf_counter() - t_up)
    upload_s = upload[-1]
    out = plan.allocate_output()
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    t = time_decode(plan, ws, out, err, args.steps, args.warmup, torch)
    exact = check_exact(plan, out, s, err, np)
    out_bytes = spec.n_symbols * spec.symbol_bytes
    alg_bytes = algorithmic_bytes(spec, info, shape.runs)
    value = out_bytes / (t["ms_per_step"] * 1e-3) / 1e9
    achieved = alg_bytes / (t["kernel_ms_mean"] * 1e-3) / 1e9
    log(f"W={lanes}: {t['ms_per_step']:.4f} ms/step, {value:.1f} GB/s decoded, exact={exact}")
    result = {
        "value": value, "ms_per_step": t["ms_per_step"], "exact": exact,
        "kernel_ms_mean": t["kernel_ms_mean"], "kernel_ms_median": t["kernel_ms_median"],
        "kernel_ms_min": t["kernel_ms_min"], "settle_launches": t["settle_launches"],
        "alg_bytes": alg_bytes, "achieved_gbs": achieved, "blob_info": info, "plan": plan,
        "blob": blob, "symbols": s, "spec": spec, "upload_s": upload_s, "upload_cold_s": upload[0],
        "upload_bytes": plan.device_bytes,
        "pcie_inclusive_gbs": out_bytes / (upload_s + t["kernel_ms_mean"] * 1e-3) / 1e9,
        "shape": {"blocks": shape.blocks, "waves_per_block": shape.waves_per_block,
                  "units_per_run": shape.units_per_run, "runs": shape.runs, "units_per_wave": shape.units_per_wave},
    }
    if not args.no_extras:
        cold = time_cold(plan, ws, out, err, torch)
        cold["hbm_frac"] = round(alg_bytes / (cold["median_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        result["cache_cold"] = cold
        log(f"W={lanes} after evicting the caches: {result['cache_cold']['median_ms']:.4f} ms")
    if not args.no_extras and shape.units_per_run != 1:
        # The same decode using every split point (one run per unit).
        kg = int(args.shape.split(",")[1]) if args.shape else 8
        plan.set_tuning(waves=shape.waves_per_block, chunk_groups=kg, units_per_run=1)
        one = plan.shape()
        t1 = time_decode(plan, ws, out, err, args.steps, args.warmup, torch)
        ok1 = check_exact(plan, out, s, err, np)
        result["every_split_point"] = {
            "decoded_gbs": round(out_bytes / (t1["ms_per_step"] * 1e-3) / 1e9, 2),
            "ms_per_step": round(t1["ms_per_step"], 5), "kernel_ms_mean": round(t1["kernel_ms_mean"], 5),
            "exact": ok1, "runs": one.runs,
            "hbm_frac": round(algorithmic_bytes(spec, info, one.runs) / (t1["kernel_ms_mean"] * 1e-3) / 1e9
                                   / HBM_PEAK_GBS, 4)}
        log(f"W={lanes} every split point: {t1['ms_per_step']:.4f} ms/step, exact={ok1}")
        plan.set_tuning(waves=shape.waves_per_block, chunk_groups=kg, units_per_run=shape.units_per_run)
    # Keep device memory for the caller to release.
    result["_buffers"] = (ws, out, err)
    return result


def run_c0(args, torch, np, rc, synth):
    """The small correctness configuration: 1 MiB Laplace(128, 4), n = 11, W = 32, 256 splits."""
    spec = synth.c0_spec()
    s = spec.generate()
    blob = rc.encode(s, lanes=spec.lanes, quant_bits=spec.quant_bits, splits=spec.splits)
    plan = rc.Plan(blob)
    ws = plan.allocate_workspace()
    plan.upload(ws)
    out = plan.allocate_output()
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    t = time_decode(plan, ws, out, err, args.steps, args.warmup, torch)
    exact = check_exact(plan, out, s, err, np)
    gbs = len(s) / (t["ms_per_step"] * 1e-3) / 1e9
    log(f"C0: {t['ms_per_step']:.4f} ms/step, {gbs:.1f} GB/s, exact={exact}")
    sh = plan.shape()
    return {"decoded_gbs": round(gbs, 2), "ms_per_step": round(t["ms_per_step"], 5), "exact": exact,
            "splits": blob.info.splits, "metadata_bytes": blob.info.metadata_bytes, "runs": sh.runs,
            "units_per_wave": sh.units_per_wave}


def run_combined(args, base, torch, np, rc):
    rows = []
    blob, s = base["blob"], base["symbols"]
    import synth
    for target in synth.C2_TARGETS:
        b = blob.combine(target)
        info = b.info
        plan = rc.Plan(b)
        ws = plan.allocate_workspace()
        plan.upload(ws)
        out = plan.allocate_output()
        err = torch.zeros(1, dtype=torch.int32, device="cuda")
        t = time_decode(plan, ws, out, err, max(3, args.steps // 2), 2, torch)
        exact = check_exact(plan, out, s, err, np)
        gbs = len(s) / (t["ms_per_step"] * 1e-3) / 1e9
        sh = plan.shape()
        rows.append({"splits": info.splits, "runs": sh.runs, "units_per_wave": sh.units_per_wave,
                     "metadata_bytes": info.metadata_bytes,
                     "transferred_bytes": info.total_bytes, "decoded_gbs": round(gbs, 2),
                     "ms": round(t["ms_per_step"], 4), "exact": exact})
        log(f"combined to {info.splits}: meta {info.metadata_bytes} B, {gbs:.1f} GB/s, exact={exact}")
        del ws, out, err, plan, b
    return rows


def run_unpack(args, base, torch, np, rc):
    """Split metadata unpacked on the device (packed plans, Sec. 4.3 format) against
    the host planner, on one stream: host time to create the plan (the host
    planner unpacks every split point's lane records; a packed plan copies the
    packed section), metadata bytes uploaded, and the unpack kernel's duration,
    for every split point and combined to fewer units (the host planner gets the
    combined blob made beforehand). Each packed plan's records are compared word
    for word with the host planner's, and its decode checked exact."""
    blob, s = base["blob"], base["symbols"]
    M = blob.splits
    rows = []
    for target in (0, M // 4, 64, 1):
        hb = blob.combine(target) if 0 < target < M else blob
        t0 = time.perf_counter()
        hb2 = blob.combine(target) if 0 < target < M else blob
        combine_s = time.perf_counter() - t0
        del hb2
        host_s = _median_time(lambda: rc.Plan(hb), reps=5)
        packed_s = _median_time(lambda: rc.Plan(blob, packed_target=target), reps=5)
        host, packed = rc.Plan(hb), rc.Plan(blob, packed_target=target)
        ws_h = host.allocate_workspace()
        host.upload(ws_h)
        ws_p = packed.allocate_workspace()
        ws_p.fill_(0xC3)
        packed.upload(ws_p)
        torch.cuda.synchronize()
        rp, lp = packed.device_records(ws_p)
        rh, lh = host.device_records(ws_h)
        same = bool(np.array_equal(rp, rh) and np.array_equal(lp, lh))
        del ws_h
        mean_ms, med_ms = _time_launches(lambda: packed.unpack(ws_p), 50, 5, torch)
        out = packed.allocate_output()
        err = torch.zeros(1, dtype=torch.int32, device="cuda")
        packed.decode(ws_p, out, err)
        torch.cuda.synchronize()
        exact = check_exact(packed, out, s, err, np) and same
        U = packed.layout().unit_count
        rows.append({"units": U, "records_equal_host": same, "exact": exact,
                     "host_plan_ms": round(host_s * 1e3, 3), "packed_plan_ms": round(packed_s * 1e3, 3),
                     "combine_ms": round(combine_s * 1e3, 3) if hb is not blob else 0.0,
                     "host_metadata_bytes": host.metadata_device_bytes,
                     "packed_metadata_bytes": packed.metadata_device_bytes,
                     "unpack_kernel_ms_mean": round(mean_ms, 5), "unpack_kernel_ms_median": round(med_ms, 5)})
        log(f"unpack: {U} units, host plan {host_s * 1e3:.2f} ms vs packed {packed_s * 1e3:.2f} ms + kernel "
            f"{med_ms * 1e3:.1f} us, metadata {host.metadata_device_bytes} vs {packed.metadata_device_bytes} B, "
            f"exact={exact}")
        del ws_p, out, err, host, packed, hb
    return rows


def run_split_writer(args, base, torch, np, rc):
    """Host encode time of the stream with the streaming split chooser against the
    threaded split writer (same split points: containers compared byte for byte)."""
    s, spec, ref = base["symbols"], base["spec"], base["blob"].to_bytes()
    row = {"symbols": spec.n_symbols, "lanes": spec.lanes, "splits": spec.splits, "host_cores": host_cores()}
    try:
        for name, t in (("streaming", 1), ("threaded", 0)):
            rc.set_split_writer_threads(t)
            t0 = time.perf_counter()
            b = rc.encode(s, lanes=spec.lanes, quant_bits=spec.quant_bits, splits=spec.splits)
            row[f"{name}_encode_s"] = round(time.perf_counter() - t0, 3)
            row[f"{name}_identical"] = b.to_bytes() == ref
            del b
    finally:
        rc.set_split_writer_threads(0)
    rc.set_split_writer_threads(1)
    t0 = time.perf_counter()
    rc.encode(s, lanes=spec.lanes, quant_bits=spec.quant_bits, splits=1)
    row["no_splits_encode_s"] = round(time.perf_counter() - t0, 3)
    rc.set_split_writer_threads(0)
    log(f"split writer: streaming {row['streaming_encode_s']} s, threaded {row['threaded_encode_s']} s, "
        f"encode without splits {row['no_splits_encode_s']} s, identical {row['streaming_identical']}/"
        f"{row['threaded_identical']}")
    return row


def run_conventional(args, base, torch, np, rc):
    """The conventional partitioning baseline (Sec. 2.3) on the same stream: P
    independently coded sub-sequences, decoded by the same kernels (no synchronisation).
    Compared with the Recoil container combined to the same parallelism: total bytes
    (what a client receives) and decoded GB/s."""
    s, recoil_blob, spec = base["symbols"], base["blob"], base["spec"]
    rows = []
    for P in (65536, 16384, 2176, 256, 16):   # 2176 and 16: the Large and Small variations of Tables 5-6
        b = rc.encode_partitioned(s, lanes=spec.lanes, quant_bits=spec.quant_bits, partitions=P)
        info = b.info
        plan = rc.Plan(b)
        ws = plan.allocate_workspace()
        plan.upload(ws)
        out = plan.allocate_output()
        err = torch.zeros(1, dtype=torch.int32, device="cuda")
        t = time_decode(plan, ws, out, err, max(3, args.steps // 2), 2, torch)
        exact = check_exact(plan, out, s, err, np)
        rb = recoil_blob if P >= recoil_blob.info.splits else recoil_blob.combine(P)
        row = {"partitions": info.splits, "container_bytes": info.total_bytes,
               "recoil_container_bytes": rb.info.total_bytes, "recoil_splits": rb.info.splits,
               "saved_by_recoil_bytes": info.total_bytes - rb.info.total_bytes,
               "decoded_gbs": round(len(s) / (t["ms_per_step"] * 1e-3) / 1e9, 2),
               "ms": round(t["ms_per_step"], 4), "exact": exact}
        rows.append(row)
        log(f"conventional P={info.splits}: {info.total_bytes} B (Recoil {rb.info.total_bytes} B at "
            f"{rb.info.splits} splits), {row['decoded_gbs']} GB/s, exact={exact}")
        del ws, out, err, plan, b
    return rows


def run_wide(args, base, torch, np, rc):
    """n = 16 (Table 3's largest quantisation level; the paper's n = 16 columns):
    the headline stream coded at n = 16 with the same split count, decoded through
    the two-level LDS table (two table reads per symbol). Container bytes against
    the n = 12 coding, decoded GB/s, exactness and the roofline position."""
    s, spec, b12 = base["symbols"], base["spec"], base["blob"]
    blob = rc.encode(s, lanes=spec.lanes, quant_bits=16, splits=spec.splits)
    info = blob.info
    plan = rc.Plan(blob)
    ws = plan.allocate_workspace()
    plan.upload(ws)
    out = plan.allocate_output()
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    t = time_decode(plan, ws, out, err, args.steps, args.warmup, torch)
    exact = check_exact(plan, out, s, err, np)
    sh = plan.shape()
    alg = (spec.n_symbols * spec.symbol_bytes + 2 * info.n_words + sh.runs * (20 + 4 * info.lanes)
           + (4 << 12) + 8 * 256)
    gbs = spec.n_symbols * spec.symbol_bytes / (t["ms_per_step"] * 1e-3) / 1e9
    log(f"n=16 W={spec.lanes}: {t['ms_per_step']:.4f} ms/step, {gbs:.1f} GB/s, {info.total_bytes} B "
        f"(n=12: {b12.info.total_bytes} B), exact={exact}")
    row = {"decoded_gbs": round(gbs, 2), "ms_per_step": round(t["ms_per_step"], 5), "exact": exact,
           "container_bytes": info.total_bytes, "n12_container_bytes": b12.info.total_bytes,
           "launch": {"blocks": sh.blocks, "waves_per_block": sh.waves_per_block, "units_per_run": sh.units_per_run,
                      "runs": sh.runs, "units_per_wave": sh.units_per_wave},
           "roofline": roofline(f"decode_units_c1_w{spec.lanes}_n16", "decode_units", alg, t["kernel_ms_mean"])}
    del ws, out, err, plan, blob
    return row


def run_adaptive(args, torch, np, rc, synth):
    """Adaptive coding (Sec. 3.1; the paper's image latents, Sec. 5.1, stand-in): 128 Mi
    uint8 symbols over 64 values, each drawn from one of 16 Laplace tables chosen by a
    per-symbol index (blocks of 256 with jitter), n = 9, W = 32, 32768 splits. Decoded
    with recoil_decode_adaptive, and the same symbols coded with one static table for
    comparison (container bytes, decoded GB/s)."""
    n_sym, T, A, nbits, W, M = 1 << 27, 16, 64, 9, 32, 32768
    t0 = time.perf_counter()
    pmfs, tidx, s = synth.adaptive_stream(6, n_sym, T, A)
    tabs = np.stack([rc.quantize((pmf * (1 << 30)).astype(np.uint64) + 1, nbits) for pmf in pmfs])
    blob_a = rc.encode_adaptive(s, tabs, tidx, lanes=W, quant_bits=nbits, splits=M, alphabet=A)
    blob_s = rc.encode(s, lanes=W, quant_bits=nbits, splits=M, alphabet=A)
    log(f"adaptive: generated and encoded {n_sym} symbols in {time.perf_counter() - t0:.1f}s")
    d_tidx = torch.from_numpy(tidx).to("cuda")
    rows = {}
    for name, blob in (("adaptive", blob_a), ("static", blob_s)):
        plan = rc.Plan(blob)
        ws = plan.allocate_workspace()
        plan.upload(ws)
        out = plan.allocate_output()
        err = torch.zeros(1, dtype=torch.int32, device="cuda")
        if name == "adaptive":
            fn = lambda: plan.decode_adaptive(ws, d_tidx, out, err)
        else:
            fn = lambda: plan.decode(ws, out, err)
        mean, med = _time_launches(fn, max(5, args.steps // 2), 2, torch)
        exact = check_exact(plan, out, s, err, np)
        sh = plan.shape()
        info = blob.info
        # Output, bitstream, per-run records, decode tables, and (adaptive) the 1-byte index per symbol.
        alg = (n_sym + 2 * info.n_words + sh.runs * (20 + 4 * W) + (4 << nbits) * (T if name == "adaptive" else 1)
               + (n_sym if name == "adaptive" else 0))
        rows[name] = {"container_bytes": info.total_bytes, "words_bytes": 2 * info.n_words,
                      "decoded_gbs": round(n_sym / (mean * 1e-3) / 1e9, 2), "ms": round(mean, 5),
                      "ms_median": round(med, 5), "exact": exact, "runs": sh.runs,
                      "hbm_frac": round(alg / (mean * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "alg_bytes": alg}
        log(f"adaptive row {name}: {info.total_bytes} B, {rows[name]['decoded_gbs']} GB/s, exact={exact}")
        del ws, out, err, plan
    rows["config"] = (f"{n_sym} uint8 symbols over {A} values, {T} Laplace tables (scales 0.5..16) chosen per "
                      f"symbol by a seeded index (blocks of 256, jitter +-1), n={nbits}, W={W}, {M} splits; "
                      f"the index (1 B per symbol) is read by the decoder and counted in alg_bytes")
    rows["saved_bytes_vs_static"] = rows["static"]["container_bytes"] - rows["adaptive"]["container_bytes"]
    return rows


def _neff(spec, s, np):
    """Quantisation bits able to code every present symbol: max(n, ceil(log2 #present))."""
    present = int(np.count_nonzero(np.bincount(s, minlength=spec.alphabet)))
    return max(spec.quant_bits, int(np.ceil(np.log2(max(present, 2)))))


def _encode_specs(specs, rc, np, label):
    """Generate and encode every stream (threads: generation and encoding release the GIL)."""
    from concurrent.futures import ThreadPoolExecutor
    workers = max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else 8))

    def one(spec):
        s = spec.generate()
        n = _neff(spec, s, np)
        blob = rc.encode(s, lanes=spec.lanes, quant_bits=n, splits=spec.splits, alphabet=spec.alphabet)
        return s, blob

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=workers) as ex:
        res = list(ex.map(one, specs))
    total = sum(x[0].nbytes for x in res)
    log(f"{label}: generated and encoded {len(res)} streams, {total / 2**30:.2f} GiB, "
        f"in {time.perf_counter() - t0:.1f}s on {workers} threads")
    return res


def _time_launches(fn, steps, warmup, torch):
    settle(fn, torch)
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    per = sorted(a.elapsed_time(b) for a, b in ev)
    return sum(per) / len(per), per[len(per) // 2]


def _batch_record_bytes(info, tuning):
    """Per stream of a batched decode: each run's records and table bytes, as in
    algorithmic_bytes. A stream's run is the tuned length, shortened for a stream
    too small to give every unit slot of a workgroup a run of that length."""
    M = max(info.splits, 1)
    slots = tuning.waves * (2 if info.lanes == 32 else 1)
    run = max(1, min(max(tuning.units_per_run, 1), -(-M // slots), M))
    runs = -(-M // run)
    table = (4 if info.symbol_bytes == 1 else 8) << info.quant_bits
    return runs * (20 + 4 * info.lanes) + table


def run_c3(args, torch, np, rc, synth):
    """Mixed batch: one graph replay of the persistent batched kernel against one
    single-stream launch per stream, both checked on every stream."""
    from paper_2306_12141_amd.batch import Batch
    specs = synth.c3_specs(args.c3_streams)
    streams = _encode_specs(specs, rc, np, "C3")
    blobs = [b for _, b in streams]
    out_bytes = sum(s.nbytes for s, _ in streams)
    words_bytes = sum(2 * b.info.n_words for b in blobs)
    meta_bytes = sum(b.info.metadata_bytes for b in blobs)
    batch = Batch(blobs)
    ws, out, err = batch.allocate()
    batch.upload(ws)
    torch.cuda.synchronize()
    n_items = batch.items
    log(f"C3: {n_items} work items, workspace {batch.workspace_bytes / 2**30:.2f} GiB")
    if args.c3_tuning:
        from paper_2306_12141_amd._lib import Tuning
        v = [int(x) for x in args.c3_tuning.split(",")]
        best, best_ms = Tuning(v[0], v[1], v[2], 0, v[3]), -1.0
        batch.set_tuning(best, ws)
    else:
        best, best_ms = batch.autotune(ws, out, err, reps=3)
    shape = {"waves": best.waves, "chunk_groups": best.chunk_groups, "pairs_per_wave": best.pairs_per_wave,
             "units_per_run": best.units_per_run}
    log(f"C3: {'set' if args.c3_tuning else 'autotuned'} {shape} ({best_ms:.3f} ms)")
    graph = batch.graph(ws, out, err)
    stream = torch.cuda.current_stream()

    def all_exact():
        torch.cuda.synchronize()
        host = out.cpu().numpy()
        ok = int(err.item()) == 0
        bad = 0
        for i, (s, _) in enumerate(streams):
            off, n = batch.output_range(i)
            if not np.array_equal(host[off:off + n].view(s.dtype), s):
                bad += 1
        return ok and bad == 0, bad

    out.fill_(0x5A)
    g_mean, g_med = _time_launches(lambda: graph.launch(stream), args.steps, args.warmup, torch)
    exact_batched, bad_b = all_exact()
    out.fill_(0xA5)
    ps_steps = max(3, args.steps // 4)
    if args.c3_batched_only:
        p_mean = p_med = float("nan")
        exact_ps, bad_p = True, 0
    else:
        p_mean, p_med = _time_launches(lambda: batch.decode_per_stream(ws, out, err), ps_steps, 1, torch)
        exact_ps, bad_p = all_exact()
    value = out_bytes / (g_mean * 1e-3) / 1e9
    per_stream = out_bytes / (p_mean * 1e-3) / 1e9
    log(f"C3: batched {value:.1f} GB/s ({g_mean:.3f} ms), per-stream {per_stream:.1f} GB/s ({p_mean:.3f} ms), "
        f"exact {exact_batched}/{exact_ps} (streams differing: {bad_b}/{bad_p})")
    alg = out_bytes + words_bytes + sum(_batch_record_bytes(b.info, best) for b in blobs)
    cpu = None
    if not args.no_cpu:
        pick = list(range(0, len(streams), max(1, len(streams) // 64)))
        cpu = cpu_oracle_streams((blobs[i].to_bytes() for i in pick), np, (streams[i][0] for i in pick),
                                 f"every {max(1, len(streams) // 64)}th stream of the batch (containers from the "
                                 f"host encoder, byte-identical to the oracle's)")
        log(f"C3 cpu oracle: {cpu['value']} GB/s")
    del ws, out, err, graph, batch
    return {
        "value": round(value, 3), "unit": "GB/s", "ms_per_step": round(g_mean, 5), "steps": args.steps,
        "warmup": args.warmup, "exact": exact_batched and exact_ps, "dtype": "u32",
        "config": {"workload": f"{len(streams)} mixed streams, 4 KiB-16 MiB log-uniform, Laplace/Zipf/uniform, "
                               f"3/4 uint8 (A=256) 1/4 uint16 (A=4096), n 10-12, W=32, ~8 KiB per split; "
                               f"one hipGraph replay of the persistent batched kernel (one launch per table class)",
                   "streams": len(streams), "decoded_bytes": out_bytes, "words_bytes": words_bytes,
                   "metadata_bytes": meta_bytes, "work_items": n_items, "tuning": shape,
                   "streams_checked": len(streams)},
        "per_stream": None if args.c3_batched_only else {
            "value": round(per_stream, 3), "unit": "GB/s", "ms": round(p_mean, 5),
            "ms_median": round(p_med, 5), "launches": len(streams), "exact": exact_ps,
            "how": "one single-stream recoil_decode launch per stream, in order, on one HIP stream"},
        "speedup_vs_per_stream": None if args.c3_batched_only else round(p_mean / g_mean, 3),
        "batched_ms_median": round(g_med, 5), "autotune_best_ms": round(best_ms, 4),
        "roofline": roofline("decode_batch_c3@" + ",".join(str(shape[k]) for k in ("waves", "chunk_groups",
                                                                                    "pairs_per_wave", "units_per_run")),
                             "decode_batch", alg, g_mean,
                             timing="mean over the timed graph replays, HIP events around each replay"),
        "cpu_baseline": cpu,
    }


LATENCY_BUCKETS = ((1, 1), (2, 7), (8, 63), (64, 511), (512, 1 << 40))


def run_c4(args, torch, np, rc, synth):
    """Serving loop at the configured Poisson load; every completed request's output is
    compared on the device with its content before the request is released."""
    import threading
    from paper_2306_12141_amd.server import Server, now_ns
    specs = synth.c4_corpus_specs(args.c4_corpus)
    corpus = _encode_specs(specs, rc, np, "C4 corpus")
    resident = sum(2 * b.info.n_words + (64 << 10) for _, b in corpus)
    resident = (resident + 255) // 256 * 256
    budget = 32 << 30
    hip_streams, max_batch, items = 4, 256, 1 << 17
    ctrl = ((256 + 2 * ((max_batch * 4 + 255) // 256 * 256) + (max_batch * 64 + 255) // 256 * 256 + items * 16)
            + 255) // 256 * 256
    arena = torch.empty(resident + hip_streams * ctrl + budget, dtype=torch.uint8, device="cuda")
    refs = [torch.from_numpy(s.view(np.uint8)).to("cuda") for s, _ in corpus]
    srv = Server(arena, resident, hip_streams=hip_streams, max_batch=max_batch, prep_threads=8,
                 items_per_launch=items)
    ids = [srv.add_content(b) for _, b in corpus]
    splits_of = [b.info.splits for _, b in corpus]
    rate, warm, dur = args.c4_rate, args.c4_warmup, args.c4_seconds
    n_req = int(rate * (warm + dur))
    arrivals = synth.poisson_arrivals(rate, n_req, seed=4)
    n_req = int(np.searchsorted(arrivals, warm + dur))
    pick = (synth.splitmix64(0xC4C4, 0, n_req) % np.uint64(len(ids))).astype(np.int64)
    want = [synth.log_uniform_int(0x5D1, i, 1, splits_of[pick[i]]) for i in range(n_req)]
    rec = {}
    verified = [0]
    vstream = torch.cuda.Stream()
    # One mismatch flag per request, set on the device by the request's comparison.
    flags = torch.zeros(n_req, dtype=torch.bool, device="cuda")
    done_evt = threading.Event()

    def poller():
        # Each completed request's output is compared with its content by kernels queued on
        # a side stream (no host synchronisation per request); the request is released once
        # an event recorded after its comparison has completed, so the comparisons pipeline
        # and releases are not held behind one another. (The completion word is written after
        # a system-scope fence that follows every store of the request, so kernels launched
        # after it is observed see the whole output.)
        from collections import deque
        waiting = deque()          # (event, request ids to release once it has completed)
        got = 0
        with torch.cuda.stream(vstream):
            while got < n_req or waiting:
                ids = []
                for c in srv.poll(timeout_us=200 if waiting else 1000):
                    got += 1
                    rec[c.tag] = (c.t_arrival_ns, c.t_admit_ns, c.t_launch_ns, c.t_done_ns, c.out_bytes, c.status,
                                  c.device_error, c.splits)
                    if c.status != 0:
                        continue
                    if c.tag % args.c4_verify_every == 0:
                        out = arena[c.out_offset: c.out_offset + c.out_bytes]
                        flags[c.tag] = torch.ne(out, refs[c.content]).any()
                        verified[0] += 1
                    ids.append(c.request_id)
                if ids:
                    ev = torch.cuda.Event()
                    ev.record(vstream)
                    waiting.append((ev, ids))
                while waiting and waiting[0][0].query():
                    for rid in waiting.popleft()[1]:
                        srv.release(rid)
                if done_evt.is_set() and got < n_req and time.time() > deadline[0]:
                    break

    deadline = [float("inf")]
    # The submitter waits in sleeps only (each releases the GIL), and threads hand the GIL
    # over every 0.1 ms, so the poller (which verifies and releases every request) never
    # waits behind a spinning submitter.
    switch = sys.getswitchinterval()
    sys.setswitchinterval(1e-4)
    th = threading.Thread(target=poller, daemon=True)
    th.start()
    t0 = now_ns() + 20_000_000
    late = 0
    for i in range(n_req):
        due = t0 + int(arrivals[i] * 1e9)
        while True:
            d = due - now_ns()
            if d <= 0:
                break
            time.sleep(d * 1e-9 if d > 100_000 else 0)
        if now_ns() - due > 1_000_000:
            late += 1
        srv.submit(ids[pick[i]], want[i], tag=i, arrival_ns=due)
    done_evt.set()
    deadline[0] = time.time() + 120
    th.join()
    sys.setswitchinterval(switch)
    st = srv.stats()
    srv.close()
    lat, win_bytes, win_words = [], 0, 0
    parts = {"queue": [], "launch": [], "device": []}
    by_units = {b: [] for b in LATENCY_BUCKETS}
    t_win0, t_win1 = t0 + int(warm * 1e9), t0 + int((warm + dur) * 1e9)
    bad = 0
    last_done = t_win0
    for tag, (ta, tad, tl, td, ob, status, derr, spl) in rec.items():
        if status != 0 or derr != 0:
            bad += 1
            continue
        if ta >= t_win0:
            ms = (td - ta) * 1e-6
            lat.append(ms)
            parts["queue"].append((tad - ta) * 1e-6)
            parts["launch"].append((tl - tad) * 1e-6)
            parts["device"].append((td - tl) * 1e-6)
            win_bytes += ob
            win_words += 2 * corpus[pick[tag]][1].info.n_words
            last_done = max(last_done, td)
            for lo, hi in LATENCY_BUCKETS:
                if lo <= spl <= hi:
                    by_units[(lo, hi)].append(ms)
    lat = np.array(sorted(lat))
    span = max(t_win1, last_done) - t_win0
    sustained = win_bytes / (span * 1e-9) / 1e9
    offered = float(np.mean([corpus[pick[i]][0].nbytes for i in range(n_req)])) * rate / 1e9

    def pct(a, p):
        return round(float(np.percentile(a, p)), 3) if len(a) else None

    buckets = {}
    for (lo, hi), v in by_units.items():
        v = np.array(v)
        name = f"{lo}" if lo == hi else (f"{lo}-{hi}" if hi < (1 << 40) else f">={lo}")
        buckets[name] = {"requests": int(len(v)), "p50": pct(v, 50), "p99": pct(v, 99),
                         "max": round(float(v.max()), 3) if len(v) else None}
    torch.cuda.synchronize()
    mismatches = torch.nonzero(flags).flatten().tolist()
    exact = not mismatches and bad == 0 and len(rec) == n_req and (
        verified[0] == n_req or args.c4_verify_every > 1)
    log(f"C4: {len(rec)}/{n_req} completed, window {len(lat)} requests, p50 {pct(lat, 50)} ms, p99 {pct(lat, 99)} "
        f"ms, sustained {sustained:.2f} GB/s (offered {offered:.2f}), late submits {late}, failed {bad}, "
        f"verified {verified[0]}, mismatches {len(mismatches)}")
    cpu = None
    if not args.no_cpu:
        first = range(min(n_req, 400))
        conts = (corpus[pick[i]][1].combine(want[i]).to_bytes() for i in first)
        syms = (corpus[pick[i]][0] for i in first)
        cpu = cpu_oracle_streams(conts, np, syms, "the first requests in arrival order, each combined to its "
                                 "requested split count (host codec containers, byte-identical to the oracle's)")
        log(f"C4 cpu oracle: {cpu['value']} GB/s")
    del refs, arena, flags
    return {
        "value": round(sustained, 3), "unit": "GB/s", "exact": exact, "dtype": "u32",
        "latency_ms": {"p50": pct(lat, 50), "p90": pct(lat, 90), "p99": pct(lat, 99), "p99.9": pct(lat, 99.9),
                       "max": round(float(lat[-1]), 3) if len(lat) else None,
                       "how": "arrival (scheduled submit time) to the launcher observing the request's "
                              "completion word, requests arriving in the window"},
        "latency_by_units_requested": buckets,
        "latency_parts_ms": {k: {"p50": pct(np.array(v), 50), "p99": pct(np.array(v), 99)} for k, v in parts.items()},
        "offered_gbs": round(offered, 3),
        "config": {"workload": f"serving: Poisson {rate:g} req/s over a resident corpus of {len(corpus)} streams "
                               f"(sizes at the quantiles of log-uniform 64 KiB-64 MiB, mean "
                               f"{np.mean([s.nbytes for s, _ in corpus]) / 2**20:.2f} MiB; C3 mix; ~1 KiB per "
                               f"stored split), per-request split count log-uniform in [1, stored], combined at "
                               f"admission, 32 GiB budget, {hip_streams} HIP streams, up to {max_batch} requests "
                               f"per launch",
                   "requests": n_req, "window_s": dur, "warmup_s": warm, "requests_in_window": int(len(lat)),
                   "requests_verified": verified[0], "verify_every": args.c4_verify_every,
                   "verify": "every completed request (verify_every 1): its output range compared with its "
                             "content on the device before release (kernels on a side stream, one mismatch "
                             "flag per request, released after the comparison's event)"},
        "launches": st.launches, "requests_per_launch": round(st.requests_launched / max(1, st.launches), 2),
        "budget_peak_bytes": st.budget_peak, "late_submits": late, "failed": bad,
        "roofline": roofline("decode_batch_c4", "decode_batch", win_bytes + win_words, span * 1e-6,
                             note="sustained over the window: decoded + bitstream bytes of the window's "
                                  "requests / window span; at this load the chip is mostly idle, so this is "
                                  "the offered utilisation, not the kernel's efficiency"),
        "cpu_baseline": cpu,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--lanes", type=int, default=64, choices=(32, 64),
                    help="interleaved lanes of the headline encoding (the other is reported in extras)")
    ap.add_argument("--shape", default="", metavar="WAVES,K,BLOCKS_PER_CU[,UNITS_PER_RUN]",
                    help="launch shape of the decode kernel (default 16,8,0,0: units per run chosen at launch)")
    ap.add_argument("--workload", default="all", choices=("all", "c1", "c3", "c4", "n16"),
                    help="all (default): the headline line with c3 and c4 in it; c1: without them; "
                         "c3 / c4 / n16: that workload's own line (n16: the headline stream coded at n = 16)")
    ap.add_argument("--c3-streams", type=int, default=4096, help="streams in the batched workload")
    ap.add_argument("--c3-tuning", default="", metavar="WAVES,K,PAIRS,UNITS_PER_RUN",
                    help="batched launch shape instead of the autotuner's choice")
    ap.add_argument("--c3-batched-only", action="store_true",
                    help="skip the per-stream launches (for counter runs of the batched kernel)")
    ap.add_argument("--c4-corpus", type=int, default=128, help="resident streams in the serving corpus")
    ap.add_argument("--c4-rate", type=float, default=2000.0, help="request arrival rate (1/s)")
    ap.add_argument("--c4-seconds", type=float, default=30.0, help="measured window after warm-up (s)")
    ap.add_argument("--c4-warmup", type=float, default=5.0, help="warm-up before the window (s)")
    ap.add_argument("--c4-verify-every", type=int, default=1,
                    help="compare every k-th request's output with its content (default 1: all)")
    ap.add_argument("--no-extras", action="store_true", help="skip the W=32, every-split, combined and C0 runs")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baselines")
    ap.add_argument("--cpu-sample", type=int, default=1 << 25, help="symbols in the oracle's C1 sample")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="first run a plain device copy of BYTES (for counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the decoder runs on a single MI355X "
              "(sharding across GPUs is not built).", file=sys.stderr)
        sys.exit(2)

    import gc

    import numpy as np
    import torch

    import paper_2306_12141_amd as rc
    import synth

    torch.cuda.set_device(0)
    if args.copy_calibration:
        # A plain device copy of known size: its FETCH_SIZE / WRITE_SIZE readings scale
        # the decode kernels' counters to bytes.
        src = torch.empty(args.copy_calibration, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload in ("c3", "c4"):
        fn = run_c3 if args.workload == "c3" else run_c4
        sub = fn(args, torch, np, rc, synth)
        line = {"metric": METRIC, "value": sub["value"], "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
                "warmup": args.warmup, "ms_per_step": sub.get("ms_per_step", (sub.get("latency_ms") or {}).get("p50")),
                "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
                "data": "synthetic (seeded streams; the paper's corpora are not available)",
                "config": sub["config"], "roofline": sub["roofline"], "cpu_baseline": sub["cpu_baseline"],
                "extras": {k: v for k, v in sub.items() if k not in ("value", "unit", "config", "roofline",
                                                                   "cpu_baseline")}}
        print(json.dumps(line), flush=True)
        return
    if args.workload == "n16":
        base = run_c1(argparse.Namespace(**{**vars(args), "no_extras": True}), torch, np, rc, synth)
        row = run_wide(args, base, torch, np, rc)
        line = {"metric": METRIC, "value": row["decoded_gbs"], "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
                "warmup": args.warmup, "ms_per_step": row["ms_per_step"], "higher_is_better": True,
                "scaling": "weak", "vs_baseline": None, "dtype": "u32",
                "data": "synthetic (seeded SplitMix64 streams; the paper's corpora are not available)",
                "config": {"workload": f"single 256 MiB uint8 stream, Zipf(1.1) over a seeded permutation of 256 "
                                       f"symbols, n=16, W={args.lanes}, {base['blob_info'].splits} splits"},
                "roofline": row["roofline"], "cpu_baseline": None,
                "extras": {k: v for k, v in row.items() if k != "roofline"}}
        print(json.dumps(line), flush=True)
        return
    base = run_c1(args, torch, np, rc, synth)
    extras = {"upload": {"bytes": base["upload_bytes"], "ms": round(base["upload_s"] * 1e3, 3),
                         "first_ms": round(base["upload_cold_s"] * 1e3, 3),
                         "pcie_inclusive_decoded_gbs": round(base["pcie_inclusive_gbs"], 2)}}
    if "every_split_point" in base:
        extras["every_split_point"] = base["every_split_point"]
    if "cache_cold" in base:
        extras["cache_cold"] = base["cache_cold"]
    if not args.no_extras:
        extras["n16"] = run_wide(args, base, torch, np, rc)
        # The same stream interleaved the other way (the workload names both), and
        # the split-count sweep on the W = 32 encoding.
        other_lanes = 32 if args.lanes == 64 else 64
        other = run_c1(argparse.Namespace(**{**vars(args), "lanes": other_lanes}), torch, np, rc, synth)
        extras[f"w{other_lanes}"] = {
            "decoded_gbs": round(other["value"], 2), "ms_per_step": round(other["ms_per_step"], 4),
            "exact": other["exact"], "metadata_bytes": other["blob_info"].metadata_bytes,
            "launch": other["shape"],
            "roofline": roofline(f"decode_units_c1_w{other_lanes}", "decode_units", other["alg_bytes"],
                                 other["kernel_ms_mean"])}
        for k in ("every_split_point", "cache_cold"):
            if k in other:
                extras[f"w{other_lanes}"][k] = other[k]
        w32 = other if other_lanes == 32 else base
        extras["combined_w32"] = run_combined(args, w32, torch, np, rc)
        extras["conventional_w32"] = run_conventional(args, w32, torch, np, rc)
        extras["device_unpack_w32"] = run_unpack(args, w32, torch, np, rc)
        extras["split_writer_w32"] = run_split_writer(args, w32, torch, np, rc)
        extras["adaptive"] = run_adaptive(args, torch, np, rc, synth)
        del other, w32
        extras["c0"] = run_c0(args, torch, np, rc, synth)
    cpu = None
    if not args.no_cpu:
        cpu = cpu_oracle_baseline(base["spec"], args.cpu_sample, np)
        log(f"cpu oracle: {cpu['value']} GB/s on {cpu['cores']} threads ({cpu['timings']})")

    info = base["blob_info"]
    sh = base["shape"]
    line = {
        "metric": METRIC,
        "value": round(base["value"], 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(base["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic (seeded SplitMix64 streams; the paper's corpora are not available)",
        "config": {
            "workload": f"single 256 MiB uint8 stream, Zipf(1.1) over a seeded permutation of 256 symbols, "
                        f"n=12, W={args.lanes}, {info.splits} splits, decoded as {sh['runs']} runs of "
                        f"{sh['units_per_run']} units (Sec. 3.3 combining at launch; every split point: "
                        f"extras.every_split_point)",
            "n_symbols": info.n_symbols, "n_words": info.n_words, "splits": info.splits,
            "lanes": args.lanes, "quant_bits": info.quant_bits,
            "metadata_bytes": info.metadata_bytes, "container_bytes": info.total_bytes,
            "bit_exact": base["exact"], "launch": sh,
        },
        "roofline": roofline(
            f"decode_units_c1_w{args.lanes}", "decode_units", base["alg_bytes"], base["kernel_ms_mean"],
            timing="mean launch duration of the timed back-to-back decodes (HIP events on the launch stream)",
            clock_settle={"ms": SETTLE_MS, "launches": base["settle_launches"]},
            single_launch_ms={"median": round(base["kernel_ms_median"], 5), "min": round(base["kernel_ms_min"], 5)}),
        "cpu_baseline": cpu,
        "extras": extras,
    }
    del base
    gc.collect()
    torch.cuda.empty_cache()
    if args.workload == "all":
        line["c3"] = run_c3(args, torch, np, rc, synth)
        gc.collect()
        torch.cuda.empty_cache()
        line["c4"] = run_c4(args, torch, np, rc, synth)
        line["config"]["bit_exact_all"] = bool(line["config"]["bit_exact"] and line["c3"]["exact"]
                                               and line["c4"]["exact"])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
