#!/usr/bin/env python3
"""Recoil decode benchmark on one MI355X.

Default workload: a single 256 MiB uint8 stream, iid Zipf(s = 1.1) over a
seeded permutation of 256 symbols, n = 12, W = 32 interleaved lanes, encoded
with 65536 splits. One step is one recoil_decode of the whole stream with the
bitstream, table and metadata already resident in HBM. `value` is decoded
output bytes per second (1 GB = 1e9 B) over the timed steps.

Also reported: the same stream at W = 64, the stream combined down to 16384 /
4096 / 1024 / 256 splits (metadata and transferred bytes, GB/s), the dominant
kernel's roofline position, and the CPU oracle timed on the host cores on a
bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c1|c0|c3|c4]
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
METRIC = "decoded GB/s on 1 MI355X (batched vs per-stream launch, bit-exact); p99 latency"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in ("paper_2306_12141_amd/csrc/device/decode.hip", "paper_2306_12141_amd/csrc/device/decode.hpp"):
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(key: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they match this kernel."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    ent = rec.get(key)
    if not ent or ent.get("kernel_hash") != kernel_source_hash():
        return None
    return ent.get("bytes_per_launch")


def time_decode(plan, ws, out, err, steps, warmup, torch):
    for _ in range(warmup):
        plan.decode(ws, out, err)
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    t_all0 = torch.cuda.Event(enable_timing=True)
    t_all1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_all0.record()
    for k in range(steps):
        starts[k].record()
        plan.decode(ws, out, err)
        ends[k].record()
    t_all1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    per = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    total_ms = t_all0.elapsed_time(t_all1)
    per.sort()
    return {"ms_total": total_ms, "ms_per_step": total_ms / steps, "kernel_ms_mean": sum(per) / len(per),
            "kernel_ms_median": per[len(per) // 2], "kernel_ms_min": per[0], "wall_s": wall}


def check_exact(plan, out, symbols, err, np):
    got = plan.symbols_of(out)
    ok = bool(np.array_equal(got, symbols)) and int(err.item()) == 0
    return ok


def cpu_oracle_baseline(spec, sample_symbols: int, np):
    """The oracle, as it stands, on a bounded prefix of the same workload, all host cores."""
    import oracle
    import synth
    s = spec.generate()[:sample_symbols] if spec.n_symbols <= sample_symbols else None
    if s is None:
        sub = synth.StreamSpec(**{**spec.__dict__, "n_symbols": sample_symbols})
        s = sub.generate()
    splits = max(1, int(spec.splits * sample_symbols / spec.n_symbols))
    p = oracle.params(lanes=spec.lanes, quant_bits=spec.quant_bits, symbol_bytes=spec.symbol_bytes,
                      alphabet=spec.alphabet)
    cont = oracle.encode(s, p, splits).container()
    dec = oracle.Decoder(cont)
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    cores = max(1, min(cores, 16))
    t0 = time.perf_counter()
    out = dec.all(aligned=True, workers=cores)
    dt = time.perf_counter() - t0
    assert np.array_equal(out, s)
    return {"value": round(len(s) * spec.symbol_bytes / dt / 1e9, 4), "unit": "GB/s", "cores": cores,
            "kind": "oracle",
            "sample": f"first {len(s)} symbols of the workload, encoded by the oracle with {splits} splits; "
                      f"all {splits} decode units over {cores} std::threads; {dt:.2f} s wall"}


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
        w, k, b = (int(v) for v in args.shape.split(","))
        plan.set_tuning(waves=w, chunk_groups=k, blocks_per_cu=b)
    ws = plan.allocate_workspace()
    plan.upload(ws)
    out = plan.allocate_output()
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    t = time_decode(plan, ws, out, err, args.steps, args.warmup, torch)
    exact = check_exact(plan, out, s, err, np)
    out_bytes = spec.n_symbols * spec.symbol_bytes
    alg_bytes = out_bytes + 2 * info.n_words + plan.metadata_device_bytes + (4 << spec.quant_bits)
    value = out_bytes / (t["ms_per_step"] * 1e-3) / 1e9
    achieved = alg_bytes / (t["kernel_ms_mean"] * 1e-3) / 1e9
    log(f"W={lanes}: {t['ms_per_step']:.4f} ms/step, {value:.1f} GB/s decoded, exact={exact}")
    result = {
        "value": value, "ms_per_step": t["ms_per_step"], "exact": exact,
        "kernel_ms_mean": t["kernel_ms_mean"], "kernel_ms_median": t["kernel_ms_median"],
        "alg_bytes": alg_bytes, "achieved_gbs": achieved, "blob_info": info, "plan": plan,
        "blob": blob, "symbols": s, "spec": spec,
    }
    # Keep device memory for the caller to release.
    result["_buffers"] = (ws, out, err)
    return result


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
        rows.append({"splits": info.splits, "metadata_bytes": info.metadata_bytes,
                     "transferred_bytes": info.total_bytes, "decoded_gbs": round(gbs, 2),
                     "ms": round(t["ms_per_step"], 4), "exact": exact})
        log(f"combined to {info.splits}: meta {info.metadata_bytes} B, {gbs:.1f} GB/s, exact={exact}")
        del ws, out, err, plan, b
    return rows


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--lanes", type=int, default=32, choices=(32, 64))
    ap.add_argument("--shape", default="", metavar="WAVES,K,BLOCKS_PER_CU",
                    help="launch shape of the decode kernel (default 16,4,0)")
    ap.add_argument("--workload", default="c1", choices=("c1",))
    ap.add_argument("--no-extras", action="store_true", help="skip the W=64 and combined-split runs")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-sample", type=int, default=1 << 26, help="symbols in the oracle's sample")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="first run a plain device copy of BYTES (for counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build decodes on a single MI355X "
              "(multi-GPU sharding is described in DESIGN.md, not run).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2306_12141_amd as rc
    import synth

    torch.cuda.set_device(0)
    if args.copy_calibration:
        # A plain device copy of known size: its FETCH_SIZE / WRITE_SIZE readings scale
        # the decode kernel's counters to bytes.
        src = torch.empty(args.copy_calibration, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    base = run_c1(args, torch, np, rc, synth)
    extras = {}
    if not args.no_extras:
        extras["combined"] = run_combined(args, base, torch, np, rc)
        if args.lanes == 32:
            other = argparse.Namespace(**{**vars(args), "lanes": 64})
            r64 = run_c1(other, torch, np, rc, synth)
            extras["w64"] = {"decoded_gbs": round(r64["value"], 2), "ms_per_step": round(r64["ms_per_step"], 4),
                             "exact": r64["exact"], "metadata_bytes": r64["blob_info"].metadata_bytes,
                             "roofline_frac": round(r64["achieved_gbs"] / HBM_PEAK_GBS, 4)}
            del r64
    cpu = None
    if not args.no_cpu:
        cpu = cpu_oracle_baseline(base["spec"], args.cpu_sample, np)
        log(f"cpu oracle: {cpu['value']} GB/s on {cpu['cores']} cores")

    info = base["blob_info"]
    key = f"decode_units_c1_w{args.lanes}"
    traffic = measured_traffic(key)
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
        "data": "synthetic (seeded SplitMix64 Zipf stream; the paper's corpora are not available)",
        "config": {
            "workload": f"single 256 MiB uint8 stream, Zipf(1.1) over a seeded permutation of 256 symbols, "
                        f"n=12, W={args.lanes}, {info.splits} splits",
            "n_symbols": info.n_symbols, "n_words": info.n_words, "splits": info.splits,
            "lanes": args.lanes, "quant_bits": info.quant_bits,
            "metadata_bytes": info.metadata_bytes, "container_bytes": info.total_bytes,
            "bit_exact": base["exact"],
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(base["achieved_gbs"], 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(base["achieved_gbs"] / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel": "decode_units",
            "alg_bytes_per_launch": base["alg_bytes"],
            "kernel_ms_mean": round(base["kernel_ms_mean"], 5),
        },
        "cpu_baseline": cpu,
        "extras": extras,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
