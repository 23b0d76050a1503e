"""Match-phase decode throughput on one MI355X.

Default workload: FASTQ-like reads, 1 GiB (whole records), 64 KiB LZ blocks,
G = 64, encoded twice -- with the base thresholds 6/8/10/12 and the tuned
12/16/24/32 (distance classes <4 KiB, <64 KiB, <1 MiB, >=1 MiB) -- and decoded
from device-resident archives into a device buffer.  A step is one full
decode of one archive; `value` is the tuned archive's output GB/s (10^9
output bytes per second), the base archive is timed the same way and both
ratios are reported.  Also: `--workload sweep` runs the match-length sweep
(256 MiB generated streams, mean match length 32..1024).

Prints one JSON line (rank 0).  Single GPU only.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    """Progress on stderr (the JSON result line goes to stdout)."""
    print("[bench %7.1fs] %s" % (time.perf_counter() - T_START, msg), file=sys.stderr, flush=True)


T_START = time.perf_counter()


def header_counts(arc):
    h = np.frombuffer(arc[:128].tobytes(), dtype=np.uint64)
    return {"n_tok": int(h[4]), "n_x16": int(h[5]), "n_x32": int(h[6]), "n_lit": int(h[7])}


def algorithmic_bytes(arc, info):
    """Bytes the method must move per decode: every output byte written once,
    every match byte and literal byte read once, every token header, length
    extension and source offset read once, plus the block table."""
    c = header_counts(arc)
    src_w = 5 if info["n"] > 0xFFFFFFFF else 4
    tok_bytes = c["n_tok"] * (1 + src_w) + 2 * c["n_x16"] + 4 * c["n_x32"] + 32 * (info["n_blocks"] + 1)
    return info["n"] + info["match_bytes"] + c["n_lit"] + tok_bytes, tok_bytes


def time_decode(torch, da, out, G, U, sched, warmup, steps):
    for _ in range(warmup):
        da.decode_async(out, G=G, unroll=U, schedule=sched)
    da.check()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record()
        da.decode_async(out, G=G, unroll=U, schedule=sched)
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    da.check()
    ms = [a.elapsed_time(b) for a, b in ev]
    return float(np.mean(ms)), float(np.median(ms)), wall


def time_stages(torch, da, out, G, U, sched, steps):
    """Parse launch and match passes timed apart (HIP events on the stream that
    launches them, i.e. torch's current stream)."""
    st = torch.cuda.current_stream()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    for a, b, c in ev:
        a.record(st)
        da.decode_stage(out, 1, G=G, unroll=U, schedule=sched)
        b.record(st)
        da.decode_stage(out, 2, G=G, unroll=U, schedule=sched)
        c.record(st)
    torch.cuda.synchronize()
    da.check()
    parse = float(np.mean([a.elapsed_time(b) for a, b, c in ev]))
    match = float(np.mean([b.elapsed_time(c) for a, b, c in ev]))
    return parse, match


def source_digest():
    import hashlib
    h = hashlib.sha256()
    for f in ("lz_device.hip", "lz_internal.h", "lz_host.cpp"):
        with open(os.path.join(ROOT, "paper_2607_18541_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


TRAFFIC_JSON = os.path.join(ROOT, "profiles", "traffic_fastq1g.json")


def measured_traffic(kernels):
    """HBM bytes per decode moved by `kernels` (all their launches), from the
    committed counter summary, if that was taken from the current kernel
    source (else None)."""
    if not os.path.exists(TRAFFIC_JSON):
        return None
    with open(TRAFFIC_JSON) as fh:
        t = json.load(fh)
    if t.get("source_sha256") != source_digest():
        return None
    got = [t.get("kernels", {}).get(k) for k in kernels]
    if got[0] is None:
        return None
    return int(sum(k["traffic_bytes_per_decode"] for k in got if k))


def traffic_from_counters(fetch_csv, write_csv, steps, n, command, depth_passes=1):
    """Writes the traffic summary from two rocprofv3 --pmc runs of
    `bench.py --profile-run` (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch).
    Each counter is scaled by what it reads for the calibration kernel of the
    same run, which reads n bytes and writes n bytes."""
    import csv
    import re

    def per_kernel(path):
        acc = {}
        for r in csv.DictReader(open(path)):
            name = r["Kernel_Name"]
            m = re.search(r"k_lz<(\d+), (\d+), (\d+), (true|false)>", name)
            key = "k_lz<%s, %s, %s, %s>" % m.groups() if m else ("calibration" if "bitwise_not" in name else None)
            if key is None:
                continue
            a = acc.setdefault(key, [0, 0.0])
            a[0] += 1
            a[1] += float(r["Counter_Value"]) * 1024.0
        return acc
    fetch, write = per_kernel(fetch_csv), per_kernel(write_csv)
    fs = n / fetch["calibration"][1]
    ws = n / write["calibration"][1]
    kernels = {}
    for k in fetch:
        if k == "calibration" or k not in write:
            continue
        kernels[k] = {"launches_per_decode": fetch[k][0] / steps,
                      "fetch_bytes_per_decode": round(fetch[k][1] * fs / steps),
                      "write_bytes_per_decode": round(write[k][1] * ws / steps),
                      "traffic_bytes_per_decode": round((fetch[k][1] * fs + write[k][1] * ws) / steps)}
    out = {"source_sha256": source_digest(),
           "workload": "FASTQ-like 1 GiB, 12/16/24/32, %d depth-aware encoder passes" % depth_passes, "steps": steps,
           "fetch_scale": round(fs, 4), "write_scale": round(ws, 4), "command": command, "kernels": kernels}
    with open(TRAFFIC_JSON, "w") as fh:
        json.dump(out, fh, indent=1)
    return out


def cpu_oracle_time(arc, n, min_s=10.0):
    """The oracle's sequential decode of the whole archive, repeated until at
    least min_s seconds of CPU time (single thread)."""
    import oracle
    reps, total = 0, 0.0
    out = None
    while total < min_s:
        t0 = time.perf_counter()
        out = oracle.decode(arc)
        total += time.perf_counter() - t0
        reps += 1
    return total / reps, reps, out


def cpu_levels_time(arc, x, min_s=3.0):
    """The level-parallel CPU decode (all host cores; tokens and depths
    prepared outside the timer, as the device plan is), repeated for at least
    min_s seconds; checked equal to the input."""
    import oracle
    prep = oracle.levels_prepare(arc)
    out = np.zeros(prep["n"], dtype=np.uint8)
    reps, total, threads = 0, 0.0, 1
    while total < min_s:
        t0 = time.perf_counter()
        threads = oracle.decode_levels_omp(prep, out)
        total += time.perf_counter() - t0
        reps += 1
    if not np.array_equal(out, x):
        raise SystemExit("level-parallel CPU decode differs from the input")
    return total / reps, reps, threads, prep["max_depth"]


def copy_ceiling(torch, n, steps):
    """Device-to-device copy of n bytes (reads n, writes n): the plain streaming
    ceiling the decode's algorithmic rate is also set against."""
    a = torch.empty(n, dtype=torch.uint8, device="cuda:0").fill_(1)
    b = torch.empty_like(a)
    b.copy_(a)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(steps):
        b.copy_(a)
    e1.record(st)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / steps
    del a, b
    torch.cuda.empty_cache()
    return 2 * n / (ms * 1e-3) / 1e9


ENTROPY_PART_NAMES = ("cmd", "x16", "x32", "src_lo_planes", "lit", "header_and_table", "src_hi_plane")


def entropy_parts(parts):
    return {k: int(round(float(v))) for k, v in zip(ENTROPY_PART_NAMES, parts)}


def entropy_stage(args, torch, lz, arc, x):
    """The paper's full pipeline on the tuned archive: tile-rANS coded
    container resident on the device, entropy stage (one wave per 64 KiB
    tile) then the match phase.  The coded ratio is the real one; the stage
    is timed apart and with the match phase (HIP events on the launching
    stream), the output checked equal to the input."""
    dev = torch.device("cuda:0")
    n = int(x.size)
    t0 = time.perf_counter()
    coded = lz.entropy_encode(arc)
    enc_s = time.perf_counter() - t0
    info = lz.entropy_info(coded)
    da = lz.DeviceArchive(coded, device=dev, coded=True)
    out = torch.empty(n, dtype=torch.uint8, device=dev)
    xt = torch.from_numpy(x).to(dev)
    st = torch.cuda.current_stream()
    for _ in range(args.warmup):
        da.entropy_decode_async()
        da.decode_async(out, G=args.G, unroll=args.unroll, schedule=args.schedule)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    for a, b, c in ev:
        a.record(st)
        da.entropy_decode_async()
        b.record(st)
        da.decode_async(out, G=args.G, unroll=args.unroll, schedule=args.schedule)
        c.record(st)
    torch.cuda.synchronize()
    da.check()
    if not bool(torch.equal(out, xt)):
        raise SystemExit("entropy stage + match phase: output differs from the input")
    ent_ms = float(np.mean([a.elapsed_time(b) for a, b, c in ev]))
    pipe_ms = float(np.mean([a.elapsed_time(c) for a, b, c in ev]))
    res = {"coded_bytes": int(coded.size), "container_bytes": int(arc.size), "ratio_coded": round(n / coded.size, 4),
           "tiles": info, "encode_s": round(enc_s, 2), "entropy_ms": round(ent_ms, 4),
           "entropy_gbps_of_container": round(arc.size / ent_ms / 1e6, 2), "pipeline_ms": round(pipe_ms, 4),
           "pipeline_gbps": round(n / pipe_ms / 1e6, 2), "entropy_share": round(ent_ms / pipe_ms, 4),
           "device_bytes": int(da.device_bytes), "bit_exact": True}
    log("entropy stage: %s" % json.dumps(res))
    da.close()
    del out, xt
    torch.cuda.empty_cache()
    return res


def sweep_points(args, torch, lz, ms=(256, 1024), log2_bs=14):
    """Generated streams of the granularity sweep (Table II method) at the
    mean match lengths where the bandwidth target is set: 256 MiB, 16 KiB
    blocks, G = 64.  Each point's cpu_baseline is the oracle's sequential
    execution of the same tokens on one host core, whose output is also the
    reference the GPU decode is compared with, byte by byte."""
    import synth
    import oracle
    dev = torch.device("cuda:0")
    n = 1 << 28
    pts = []
    for i, m in enumerate((32, 64, 128, 256, 512, 1024)):
        if m not in ms:
            continue
        ll, ml, sr, lit = synth.geo_tokens(n, m, seed=2 + i)
        t0 = time.perf_counter()
        ref = oracle.exec_tokens(n, ll, ml, sr, lit)
        cpu_s = time.perf_counter() - t0
        arc = lz.build_archive(n, log2_bs, ll, ml, sr, lit)
        info = lz.archive_info(arc)
        alg, _ = algorithmic_bytes(arc, info)
        da = lz.DeviceArchive(arc, device=dev)
        out = torch.empty(n, dtype=torch.uint8, device=dev)
        mean_ms, _, _ = time_decode(torch, da, out, 64, args.unroll, args.schedule, args.warmup, args.steps)
        if not bool(torch.equal(out, torch.from_numpy(ref).to(dev))):
            raise SystemExit("generated stream m=%d: GPU decode differs from the oracle" % m)
        parse_ms, match_ms = time_stages(torch, da, out, 64, args.unroll, args.schedule, args.steps)
        match_alg = 2 * (info["match_bytes"] - da.fused_bytes)
        pt = {"m": m, "n_bytes": n, "log2_bs": log2_bs, "G": 64, "realized_m": round(info["mean_match"], 1),
              "depths": da.levels, "fused_matches": da.fused, "ms": round(mean_ms, 4), "gbps": round(n / mean_ms / 1e6, 2),
              "alg_gbps": round(alg / mean_ms / 1e6, 2), "frac": round(alg / mean_ms / 1e6 / HBM_PEAK_GBS, 4),
              "match_stage": {"ms": round(match_ms, 4), "alg_gbps": round(match_alg / match_ms / 1e6, 2),
                              "frac": round(match_alg / match_ms / 1e6 / HBM_PEAK_GBS, 4)},
              "parse_ms": round(parse_ms, 4), "oracle_checked": True,
              "cpu_baseline": {"value": round(n / cpu_s / 1e9, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
                               "sample": "sequential execution of the whole stream's tokens, one run"}}
        log("sweep point: %s" % json.dumps(pt))
        pts.append(pt)
        da.close()
        del out
        torch.cuda.empty_cache()
    return pts


def achieved_all(t):
    return t["alg_bytes"] / (t["mean_ms"] * 1e-3) / 1e9


def capped_point(args, torch, lz, x, cap):
    """12/16/24/32 encoded with the encoder's depth cap: the matches that would
    lie deeper than `cap` become literals; decode time, depths and both ratios,
    the output checked equal to the input."""
    dev = torch.device("cuda:0")
    n = int(x.size)
    log("encoding 12/16/24/32 with depth cap %d" % cap)
    arc = lz.encode(x, args.log2_bs, lz.TUNED_THR, lz.BOUNDS_CFG, max_chain=args.max_chain,
                    depth_passes=args.depth_passes, depth_cap=cap)
    ent, _ = lz.entropy_size(arc)
    info = lz.archive_info(arc)
    da = lz.DeviceArchive(arc, device=dev)
    out = torch.empty(n, dtype=torch.uint8, device=dev)
    mean_ms, _, _ = time_decode(torch, da, out, args.G, args.unroll, args.schedule, args.warmup, args.steps)
    if not bool(torch.equal(out, torch.from_numpy(x).to(dev))):
        raise SystemExit("depth cap %d: GPU decode differs from the input" % cap)
    pt = {"depth_cap": cap, "depths": da.levels, "ms": round(mean_ms, 4), "gbps": round(n / mean_ms / 1e6, 3),
          "ratio_raw": round(n / arc.size, 4), "ratio_entropy": round(n / ent, 4),
          "coverage": round(info["coverage"], 4), "bit_exact": True}
    log("depth cap point: %s" % json.dumps(pt))
    da.close()
    del out
    torch.cuda.empty_cache()
    return pt


def run_fastq(args, torch, lz):
    import synth
    dev = torch.device("cuda:0")
    # the generated-stream points first: timed after the FASTQ work in the
    # same process they came out 10-15 % slower than in a process of their own
    points = None if args.no_sweep_points else sweep_points(args, torch, lz)
    t0 = time.perf_counter()
    log("generating %d B of FASTQ-like reads" % args.size)
    x = synth.fastq(args.size, seed=3)
    n = int(x.size)
    gen = {"gen_s": round(time.perf_counter() - t0, 2)}
    log("generated %d B" % n)
    res = {}
    for name, thr in (("base", lz.BASE_THR), ("tuned", lz.TUNED_THR)):
        t0 = time.perf_counter()
        log("encoding %s %s" % (name, thr))
        arc = lz.encode(x, args.log2_bs, thr, lz.BOUNDS_CFG, max_chain=args.max_chain, depth_passes=args.depth_passes)
        enc_s = time.perf_counter() - t0
        log("encoded %s: %d B archive in %.1fs" % (name, arc.size, enc_s))
        info = lz.archive_info(arc)
        ent, parts = lz.entropy_size(arc)
        t0 = time.perf_counter()
        da = lz.DeviceArchive(arc, device=dev)
        open_s = time.perf_counter() - t0
        log("opened %s on the device in %.1fs (%d levels)" % (name, open_s, da.levels))
        out = torch.empty(n, dtype=torch.uint8, device=dev)
        mean_ms, med_ms, wall = time_decode(torch, da, out, args.G, args.unroll, args.schedule, args.warmup,
                                            args.steps)
        # bit-exact check outside the timer: device compare with the input
        ok = bool(torch.equal(out, torch.from_numpy(x).to(dev)))
        if not ok:
            raise SystemExit(f"{name}: GPU decode differs from the input")
        alg, tok_bytes = algorithmic_bytes(arc, info)
        log("decoded %s: %.3f ms per decode, %.2f GB/s, bit-exact" % (name, mean_ms, n / mean_ms / 1e6))
        parse_ms, match_ms = time_stages(torch, da, out, args.G, args.unroll, args.schedule, args.steps)
        if not bool(torch.equal(out, torch.from_numpy(x).to(dev))):
            raise SystemExit(f"{name}: staged GPU decode differs from the input")
        log("stages %s: parse %.3f ms, match passes %.3f ms" % (name, parse_ms, match_ms))
        g32_ms = None
        if name == "tuned" and args.G != 32:
            # the configuration's own cooperation width, beside the default
            g32_ms, _, _ = time_decode(torch, da, out, 32, args.unroll, args.schedule, args.warmup, args.steps)
            if not bool(torch.equal(out, torch.from_numpy(x).to(dev))):
                raise SystemExit("tuned, G=32: GPU decode differs from the input")
            log("decoded tuned at G=32: %.3f ms, %.2f GB/s" % (g32_ms, n / g32_ms / 1e6))
        res[name] = {
            "arc": arc, "info": info, "mean_ms": mean_ms, "median_ms": med_ms, "wall_s": wall,
            "gbps": n / (mean_ms * 1e-3) / 1e9, "alg_bytes": alg, "tok_bytes": tok_bytes,
            "ratio_raw": n / arc.size, "ratio_entropy": n / ent, "enc_s": enc_s, "open_s": open_s,
            "levels": da.levels, "parse_ms": parse_ms, "match_ms": match_ms, "device_bytes": da.device_bytes,
            "fused": da.fused, "fused_bytes": da.fused_bytes,
            "entropy_parts": entropy_parts(parts), "g32_ms": g32_ms,
        }
        da.close()
        del out
        torch.cuda.empty_cache()
    cap_pt = capped_point(args, torch, lz, x, 16)
    t = res["tuned"]
    b = res["base"]
    # the two kernels of a decode and their algorithmic bytes: the parse launch
    # reads the token streams and literals and writes the literals, and copies
    # the literal-sourced matches (read once, written once); the match passes
    # read and write every other match byte once
    ti = t["info"]
    parse_alg = t["tok_bytes"] + 2 * (ti["n"] - ti["match_bytes"]) + 2 * t["fused_bytes"]
    match_alg = 2 * (ti["match_bytes"] - t["fused_bytes"])
    G, U = args.G, args.unroll
    kparse = ["k_lz<%d, %d, 3, false>" % (G, U)]
    kmatch = ["k_lz<%d, %d, 1, false>" % (G, U), "k_lz<64, %d, 4, false>" % U]
    if t["parse_ms"] >= t["match_ms"]:
        dom, dom_alg, dom_ms = kparse, parse_alg, t["parse_ms"]
    else:
        dom, dom_alg, dom_ms = kmatch, match_alg, t["match_ms"]
    achieved = dom_alg / (dom_ms * 1e-3) / 1e9
    ceiling = copy_ceiling(torch, n, max(args.steps, 5))
    log("streaming copy ceiling: %.1f GB/s (read + write)" % ceiling)
    line = {
        "metric": "match-phase decode GB/s (device-resident) + ratio, 6/8/10/12 vs 12/16/24/32",
        "value": round(t["gbps"], 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t["mean_ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {
            "workload": "FASTQ-like reads %d B, 64 KiB blocks, G=%d, 12/16/24/32 (value) vs 6/8/10/12"
                        % (n, args.G),
            "n_bytes": n, "log2_bs": args.log2_bs, "G": args.G, "unroll": args.unroll,
            "schedule": args.schedule, "bounds": list(lz.BOUNDS_CFG), "max_chain": args.max_chain,
            "depth_passes": args.depth_passes,
        },
        "detail": {
            "tuned_gbps": round(t["gbps"], 3), "base_gbps": round(b["gbps"], 3),
            "tuned_ratio_raw": round(t["ratio_raw"], 4), "base_ratio_raw": round(b["ratio_raw"], 4),
            "tuned_ratio_entropy": round(t["ratio_entropy"], 4), "base_ratio_entropy": round(b["ratio_entropy"], 4),
            "tuned_mean_match": round(t["info"]["mean_match"], 2), "base_mean_match": round(b["info"]["mean_match"], 2),
            "tuned_coverage": round(t["info"]["coverage"], 4), "base_coverage": round(b["info"]["coverage"], 4),
            "tuned_levels": t["levels"], "base_levels": b["levels"],
            "tuned_parse_copied_matches": {"count": t["fused"], "bytes": t["fused_bytes"]},
            "base_ms": round(b["mean_ms"], 4), "encode_s": [round(b["enc_s"], 2), round(t["enc_s"], 2)],
            "bit_exact": True, **gen,
            "tuned_G32": {"G": 32, "ms": round(t["g32_ms"], 4), "gbps": round(n / t["g32_ms"] / 1e6, 3)}
            if t["g32_ms"] else None,
            "tuned_depth_cap16": cap_pt,
            # everything resident on the device per archive: the archive, the
            # depth plan and parse segments computed at open, and the match table
            "residency": {k: {"archive_bytes": int(res[k]["arc"].size), "device_bytes": int(res[k]["device_bytes"]),
                              "plan_and_table_bytes": int(res[k]["device_bytes"] - res[k]["arc"].size),
                              "ratio_raw": round(res[k]["ratio_raw"], 4),
                              "ratio_resident": round(n / res[k]["device_bytes"], 4)} for k in ("base", "tuned")},
            "entropy_bound_bytes_by_stream": {k: res[k]["entropy_parts"] for k in ("base", "tuned")},
        },
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(dom),
            "kernel": " + ".join(dom), "alg_bytes_per_decode": dom_alg, "ms_per_decode": round(dom_ms, 4),
            "copy_ceiling": round(ceiling, 1), "frac_of_copy": round(achieved / ceiling, 4),
        },
        "stages": {
            "parse": {"kernel": kparse[0], "ms": round(t["parse_ms"], 4), "alg_bytes": parse_alg,
                      "alg_gbps": round(parse_alg / t["parse_ms"] / 1e6, 2)},
            "match": {"kernel": " + ".join(kmatch), "ms": round(t["match_ms"], 4), "alg_bytes": match_alg,
                      "alg_gbps": round(match_alg / t["match_ms"] / 1e6, 2), "depths": t["levels"]},
            "whole_decode_alg_gbps": round(achieved_all(t), 2),
        },
    }
    line["entropy_stage"] = entropy_stage(args, torch, lz, t["arc"], x)
    if points is not None:
        line["sweep_points"] = points
    if not args.no_cpu:
        log("timing the CPU oracle decode")
        dt, reps, out = cpu_oracle_time(t["arc"], n)
        assert np.array_equal(out, x)
        line["cpu_baseline"] = {"value": round(n / dt / 1e9, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
                                "sample": "whole 12/16/24/32 archive (%d output bytes), sequential decode incl. "
                                          "validation, mean of %d runs" % (n, reps)}
        log("timing the level-parallel CPU decode")
        dt, reps, threads, depth = cpu_levels_time(t["arc"], x)
        line["cpu_parallel"] = {"value": round(n / dt / 1e9, 4), "unit": "GB/s", "cores": threads,
                                "kind": "oracle tokens, depth-parallel (OpenMP)",
                                "sample": "whole 12/16/24/32 archive, %d depths, tokens and depths prepared "
                                          "outside the timer, mean of %d runs" % (depth, reps)}
    return line


def run_profile(args, torch, lz):
    """For counter collection: the 12/16/24/32 archive decoded `steps` times,
    then one plain elementwise kernel over the n output bytes (reads n bytes,
    writes n bytes) that calibrates the memory counters."""
    import synth
    dev = torch.device("cuda:0")
    x = synth.fastq(args.size, seed=3)
    n = int(x.size)
    log("encoding")
    arc = lz.encode(x, args.log2_bs, lz.TUNED_THR, lz.BOUNDS_CFG, max_chain=args.max_chain, depth_passes=args.depth_passes)
    da = lz.DeviceArchive(arc, device=dev)
    out = torch.empty(n, dtype=torch.uint8, device=dev)
    for i in range(args.steps):
        da.decode_async(out, G=args.G, unroll=args.unroll, schedule=args.schedule)
        log("decode %d launched" % i)
    torch.cuda.synchronize()
    da.check()
    if not bool(torch.equal(out, torch.from_numpy(x).to(dev))):
        raise SystemExit("GPU decode differs from the input")
    y = torch.empty_like(out)
    torch.bitwise_not(out, out=y)
    torch.cuda.synchronize()
    return {"profile_run": True, "n": n, "steps": args.steps, "calibration": "bitwise_not over n bytes"}


def copy_units(span, G, max_bytes):
    """Token ranges for the pure-copy control: a new unit starts where the
    output offset crosses a multiple of max_bytes, and every G tokens inside
    such a stretch (so at most G tokens, about max_bytes bytes each)."""
    span = np.asarray(span, dtype=np.int64)
    T = span.size
    if T == 0:
        return np.zeros(1, dtype=np.uint64)
    bucket = (np.concatenate([[0], np.cumsum(span)[:-1]]) // max_bytes)
    first = np.concatenate([[True], bucket[1:] != bucket[:-1]])
    start_of = np.maximum.accumulate(np.where(first, np.arange(T), 0))
    cut = first | ((np.arange(T) - start_of) % G == 0)
    return np.concatenate([np.nonzero(cut)[0], [T]]).astype(np.uint64)


def run_batch(args, torch, lz):
    """Batched decode: `count` independent archives, sizes log-uniform from
    4 KiB to 16 MiB, even ones Zipf text and odd ones FASTQ-like reads,
    thresholds alternating 6/8/10/12 and 12/16/24/32.  Timed three ways: one
    decode call per archive (each its own launch sequence), one batch graph
    with the default configuration, and one batch graph with the per-bucket
    configuration the autotuner picks."""
    import synth
    dev = torch.device("cuda:0")
    k = args.count
    sizes = synth.loguniform(k, 4096, 16 << 20, 4)
    das, outs, ins = [], [], []
    total = 0
    t0 = time.perf_counter()
    for i, sz in enumerate(sizes):
        sz = int(sz)
        x = synth.zipf_text(sz, seed=4000 + i) if i % 2 == 0 else synth.fastq(sz, seed=4000 + i)
        thr = (lz.BASE_THR, lz.TUNED_THR)[(i // 2) % 2]
        arc = lz.encode(x, args.log2_bs, thr, lz.BOUNDS_CFG, max_chain=args.max_chain, depth_passes=args.depth_passes)
        da = lz.DeviceArchive(arc, device=dev)
        das.append(da)
        outs.append(torch.empty(max(da.n, 1), dtype=torch.uint8, device=dev))
        ins.append(torch.from_numpy(x).to(dev))
        total += da.n
        if (i + 1) % 256 == 0:
            log("encoded and opened %d/%d archives (%.2f GiB) in %.0fs" % (i + 1, k, total / 2**30,
                                                                       time.perf_counter() - t0))

    def check(label):
        for i, (o, x) in enumerate(zip(outs, ins)):
            if not bool(torch.equal(o[:x.numel()], x)):
                raise SystemExit("%s: archive %d differs" % (label, i))

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    res = {}
    for o in outs:
        o.fill_(0)
    ms = timed(lambda: [d.decode_async(o, G=args.G, unroll=args.unroll) for d, o in zip(das, outs)], args.steps)
    check("per-archive")
    res["per_archive"] = {"ms": round(ms, 3), "gbps": round(total / ms / 1e6, 2)}
    log("per-archive launches: %.3f ms, %.1f GB/s" % (ms, total / ms / 1e6))
    for o in outs:
        o.fill_(0)
    b = lz.Batch(das, outs, None)
    ms = timed(b.launch, args.steps)
    check("batch")
    res["batch_default"] = {"ms": round(ms, 3), "gbps": round(total / ms / 1e6, 2), "launches": b.launches}
    log("one batch graph (G=64, U=2): %.3f ms, %.1f GB/s" % (ms, total / ms / 1e6))
    b.destroy()
    cfgs, report = lz.autotune(das, outs, reps=2)
    log("autotuned %d buckets" % len(report))
    for o in outs:
        o.fill_(0)
    b = lz.Batch(das, outs, cfgs)
    ms = timed(b.launch, args.steps)
    check("batch autotuned")
    res["batch_autotuned"] = {"ms": round(ms, 3), "gbps": round(total / ms / 1e6, 2), "launches": b.launches,
                              "buckets": [{"bytes": [r["min_bytes"], r["max_bytes"]], "archives": r["archives"],
                                           "best": list(r["best"]), "best_ms": round(r["best_ms"], 4),
                                           "default_ms": round(r["default_ms"], 4)} for r in report],
                              "kept_bucket_choices": any(tuple(c)[:5] != (64, 2, 1, 0, 0) for c in cfgs)}
    log("one batch graph, autotuned: %.3f ms, %.1f GB/s" % (ms, total / ms / 1e6))
    b.destroy()
    best = max(v["gbps"] for v in res.values())
    return {"metric": "batched decode GB/s (device-resident)", "value": best, "unit": "GB/s", "n_gpus": 1,
            "steps": args.steps, "warmup": 1, "ms_per_step": res["batch_autotuned"]["ms"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
            "config": {"workload": "%d archives, log-uniform 4 KiB-16 MiB, %d B total, half Zipf text, half "
                                   "FASTQ-like, thresholds alternating" % (k, total)},
            "detail": res}


def run_serve(args, torch, lz):
    """Serving loop: Poisson arrivals of range decodes (lengths log-uniform
    16 KiB-64 MiB, offsets uniform) against one device-resident FASTQ-like
    archive, admitted by slots and arena memory; each tick launches one merged
    group per decode horizon.  Latency = submit to observed completion (host
    clock)."""
    import synth
    dev = torch.device("cuda:0")
    n = args.size
    t0 = time.perf_counter()
    x = synth.fastq(n, seed=5)
    n = int(x.size)
    log("generated %d B in %.0fs" % (n, time.perf_counter() - t0))
    seg = args.segment_mib << 20 if args.segment_mib >= 0 else ((1 << 30) if n > (3 << 30) else 0)
    arc = lz.encode(x, args.log2_bs, lz.TUNED_THR, lz.BOUNDS_CFG, max_chain=args.max_chain, depth_passes=args.depth_passes, segment=seg,
                    progress=lambda d, t: log("encoded %d of %d input bytes" % (d, t)))
    log("encoded: %d B archive (ratio %.3f) in %.0fs" % (arc.size, n / arc.size, time.perf_counter() - t0))
    da = lz.DeviceArchive(arc, device=dev)
    log("opened on the device (%d depths)" % da.levels)
    del arc
    k = args.requests
    lens = synth.loguniform(k, 16 << 10, 64 << 20, 51).astype(np.int64)
    offs = (synth.uniform(k, 52) * (n - lens)).astype(np.int64)
    # one-at-a-time service time: a few requests served one after another
    t1 = time.perf_counter()
    for i in range(8):
        da.decode_range(int(offs[i]), int(lens[i]))
    torch.cuda.synchronize()
    per_req = (time.perf_counter() - t1) / 8
    tot = int(lens.sum())

    def serve(arrive, label):
        """Requests i arrive at arrive[i] seconds; returns the level's row."""
        srv = lz.Server(da, args.arena << 20, slots=args.slots)
        lat = np.zeros(k)
        pending = {}
        nxt = 0
        done = 0
        T0 = time.perf_counter()
        last_log = T0
        while done < k:
            now = time.perf_counter() - T0
            while nxt < k and arrive[nxt] <= now:
                rid = srv.submit(int(offs[nxt]), int(lens[nxt]))
                pending[rid] = (nxt, T0 + arrive[nxt])
                nxt += 1
            srv.tick()
            for rid in srv.completed():
                i, ta = pending.pop(rid)
                lat[i] = time.perf_counter() - ta
                if srv.status(rid)[0] != 2:
                    raise SystemExit("%s: request %d failed" % (label, i))
                srv.release(rid)
                done += 1
            if time.perf_counter() - last_log > 10:
                last_log = time.perf_counter()
                log("%s: served %d/%d requests" % (label, done, k))
            if nxt < k and not pending:
                time.sleep(max(0.0, min(0.001, arrive[nxt] - (time.perf_counter() - T0))))
        wall = time.perf_counter() - T0
        hw = srv.stats()["arena_high_water"]
        max_groups = srv.stats()["max_running_groups"]
        srv.destroy()
        row = {"level": label, "served_req_per_s": round(k / wall, 2), "gbps": round(tot / wall / 1e9, 3),
               "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
               "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 2),
               "mean_ms": round(float(lat.mean()) * 1e3, 2), "wall_s": round(wall, 2), "arena_high_water": int(hw),
               "max_groups_in_flight": int(max_groups)}
        log("%s: %s" % (label, json.dumps(row)))
        return row

    def poisson(rate):
        return np.cumsum(-np.log(1.0 - synth.uniform(k, 53)) / rate)

    rows = []
    # saturated capacity: every request queued at once
    sat = serve(np.zeros(k), "saturated")
    cap = k / sat["wall_s"]
    sat["offered_req_per_s"] = None
    rows.append(sat)
    # offered loads as fractions of the saturated capacity
    for f in [float(v) for v in str(args.capacity).split(",") if v]:
        r = serve(poisson(f * cap), "%.2f of capacity" % f)
        r["offered_req_per_s"] = round(f * cap, 2)
        rows.append(r)
    # offered loads as multiples of the one-at-a-time service rate
    for load in [float(v) for v in str(args.load).split(",") if v]:
        r = serve(poisson(load / per_req), "%.1f x one-at-a-time" % load)
        r["offered_req_per_s"] = round(load / per_req, 2)
        rows.append(r)
    # every tenth request checked against the input
    for i in range(0, k, 10):
        got = da.decode_range(int(offs[i]), int(lens[i]))
        if not bool(torch.equal(got, torch.from_numpy(x[offs[i]:offs[i] + lens[i]]).to(dev))):
            raise SystemExit("range %d differs" % i)
    best = max(rows, key=lambda r: r["gbps"])
    return {"metric": "range-serving GB/s and latency", "value": best["gbps"], "unit": "GB/s",
            "n_gpus": 1, "steps": k, "warmup": 8, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "u8", "data": "synthetic",
            "config": {"workload": "FASTQ-like %d B (12/16/24/32, %s), %d range requests of 16 KiB-64 MiB per "
                                   "level: all at once (saturated), then Poisson at fractions of that capacity"
                                   % (n, "%d MiB segments" % (seg >> 20) if seg else "one segment", k),
                       "arena_mib": args.arena, "slots": args.slots},
            "detail": {"alone_ms": round(per_req * 1e3, 2), "mean_request_bytes": int(lens.mean()),
                       "capacity_req_per_s": round(cap, 2), "loads": rows, "best": best}}


def run_sweep(args, torch, lz):
    """Granularity sweep (the copy sweep of Table II): generated streams of n
    bytes whose match lengths are geometric with mean m, sources uniform over
    positions >= 64 KiB back, 1 % literal bytes.  For every m: the full decode
    for each block size and G, and the pure-copy control (every token
    independent, sources in a reference copy of the output) for each G."""
    import synth
    import oracle
    dev = torch.device("cuda:0")
    n = args.size
    rows = []
    cpu = []
    for i, m in enumerate((32, 64, 128, 256, 512, 1024)):
        ll, ml, sr, lit = synth.geo_tokens(n, m, seed=2 + i)
        # cpu_baseline leg: the oracle executes the same tokens sequentially on
        # one host core; its output is what every decode is compared with
        t0 = time.perf_counter()
        expect = torch.from_numpy(oracle.exec_tokens(n, ll, ml, sr, lit)).to(dev)
        cpu.append({"m": m, "gbps": round(n / (time.perf_counter() - t0) / 1e9, 4)})
        ref = None  # the first GPU decode (equal to the oracle's): the pure copy's source buffer
        for lb in (14, 16, 18, 20):
            arc = lz.build_archive(n, lb, ll, ml, sr, lit)
            info = lz.archive_info(arc)
            da = lz.DeviceArchive(arc, device=dev)
            out = torch.empty(n, dtype=torch.uint8, device=dev)
            alg, _ = algorithmic_bytes(arc, info)
            for G in (8, 16, 32, 64):
                mean_ms, med_ms, wall = time_decode(torch, da, out, G, args.unroll, args.schedule, 2, args.steps)
                if not bool(torch.equal(out, expect)):
                    raise SystemExit("decode differs from the oracle (m=%d log2_bs=%d G=%d)" % (m, lb, G))
                if ref is None:
                    ref = out.clone()
                rows.append({"mode": "decode", "m": m, "log2_bs": lb, "G": G, "lanes": G * info["n_blocks"],
                             "gbps": round(n / mean_ms / 1e6, 2), "alg_gbps": round(alg / mean_ms / 1e6, 2),
                             "frac": round(alg / mean_ms / 1e6 / HBM_PEAK_GBS, 4), "depths": da.levels,
                             "realized_m": round(info["mean_match"], 1)})
                log(json.dumps(rows[-1]))
            da.close()
            del out
        # pure-copy control on the same tokens
        T = len(ll)
        llv = np.asarray(ll, dtype=np.int64)
        mlv = np.asarray(ml, dtype=np.int64)
        dst = np.concatenate([[0], np.cumsum(llv + mlv)[:-1]]).astype(np.uint64)
        loff = np.concatenate([[0], np.cumsum(llv)[:-1]]).astype(np.uint64)
        g = lambda a, dt: torch.from_numpy(np.ascontiguousarray(np.asarray(a).astype(dt))).to(dev)
        tdst, tlo, tll, tsrc, tml = g(dst, np.uint64), g(loff, np.uint64), g(llv, np.uint32), g(sr, np.uint64), \
            g(mlv, np.uint32)
        tlit = g(lit, np.uint8)
        out = torch.empty(n, dtype=torch.uint8, device=dev)
        pc_alg = n + int(mlv.sum()) + int(llv.sum()) + T * 28
        for G in (8, 16, 32, 64):
            us = g(copy_units(llv + mlv, G, 2048), np.uint64)
            pc = lz.PureCopy(tdst, tlo, tll, tsrc, tml, us, tlit, ref, out)
            pc.run(G=G, unroll=args.unroll)
            torch.cuda.synchronize()
            if not bool(torch.equal(out, expect)):
                raise SystemExit("pure copy differs from the oracle (m=%d G=%d)" % (m, G))
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(args.steps):
                pc.run(G=G, unroll=args.unroll)
            b.record()
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / args.steps
            rows.append({"mode": "purecopy", "m": m, "G": G, "gbps": round(n / ms / 1e6, 2),
                         "alg_gbps": round(pc_alg / ms / 1e6, 2), "frac": round(pc_alg / ms / 1e6 / HBM_PEAK_GBS, 4)})
            log(json.dumps(rows[-1]))
        del out, ref, expect
        torch.cuda.empty_cache()
    best = max(r["gbps"] for r in rows if r["mode"] == "decode" and r["m"] >= 256)
    best_frac = max(r["frac"] for r in rows if r["mode"] == "decode" and r["m"] >= 256)
    return {"metric": "match-phase decode GB/s vs mean match length", "value": best, "unit": "GB/s",
            "n_gpus": 1, "steps": args.steps, "warmup": 2, "ms_per_step": None, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
            "config": {"workload": "match-length sweep, %d B streams, m in 32..1024, 16 KiB-1 MiB blocks, "
                                   "G in 8..64" % n},
            "best_frac_m_ge_256": best_frac, "rows": rows,
            "cpu_baseline": {"value": min(c["gbps"] for c in cpu), "unit": "GB/s", "cores": 1, "kind": "oracle",
                             "sample": "sequential execution of each m's whole %d-byte token stream, one run per m "
                                       "(per m: %s)" % (n, json.dumps(cpu))}}


def run_seek(args, torch, lz):
    """Latency of one range decode (a seek) on the device-resident
    12/16/24/32 FASTQ-like archive, by offset and length: host plan time,
    device time (events on the launching stream) and their sum, with the plan
    mode (token closure, or a device prefix decode when the closure exceeds
    its budget)."""
    import synth
    dev = torch.device("cuda:0")
    x = synth.fastq(args.size, seed=3)
    n = int(x.size)
    seg = max(args.segment_mib, 0) << 20
    arc = lz.encode(x, args.log2_bs, lz.TUNED_THR, lz.BOUNDS_CFG, max_chain=args.max_chain, depth_passes=args.depth_passes, segment=seg)
    da = lz.DeviceArchive(arc, device=dev)
    rows = []
    st = torch.cuda.current_stream()
    for length in (16384, 1 << 20):
        for frac in (0.0001, 0.001, 0.01, 0.1, 0.5, 0.99):
            off = min(int(frac * n), n - length)
            best = None
            for rep in range(args.steps):
                t0 = time.perf_counter()
                plan = da.range_plan([off], [length])
                t_plan = time.perf_counter() - t0
                out = torch.empty(length, dtype=torch.uint8, device=dev)
                scratch = torch.empty(max(plan.scratch_bytes, 1), dtype=torch.uint8, device=dev)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                t1 = time.perf_counter()
                e0.record(st)
                plan.run(out, [0], scratch)
                e1.record(st)
                e1.synchronize()
                t_run = time.perf_counter() - t1
                dev_ms = e0.elapsed_time(e1)
                if rep == 0 and not np.array_equal(out.cpu().numpy(), x[off:off + length]):
                    raise SystemExit("seek off=%d len=%d differs from the input" % (off, length))
                row = {"len": length, "off": off, "frac": frac, "plan_ms": round(t_plan * 1e3, 3),
                       "device_ms": round(dev_ms, 3), "total_ms": round((t_plan + t_run) * 1e3, 3),
                       "mode": "prefix" if plan.prefix_bytes else "closure",
                       "closure_bytes": plan.closure_bytes, "prefix_bytes": plan.prefix_bytes,
                       "horizon": plan.horizon,
                       "depths": plan.levels}
                if best is None or row["total_ms"] < best["total_ms"]:
                    best = row
                plan.free()
                del scratch, out
            log(json.dumps(best))
            rows.append(best)
    # read-level seek (record id -> block -> record), FASTQ records of 4 lines
    idx = lz.ReadIndex(x, args.log2_bs, 4)
    out = torch.empty(1 << 16, dtype=torch.uint8, device=dev)
    scratch = torch.empty(64 << 20, dtype=torch.uint8, device=dev)
    R = idx.records
    rec_rows = []
    for frac in (0.0001, 0.01, 0.1, 0.5, 0.99):
        rid = min(int(frac * R), R - 1)
        best = None
        for rep in range(args.steps):
            t0 = time.perf_counter()
            got = idx.seek(da, rid, out=out, scratch=scratch)
            ms = (time.perf_counter() - t0) * 1e3
            best = ms if best is None else min(best, ms)
        rec = bytes(got.cpu().numpy())
        # the record is 4 lines and its header names its id (ids count from 1)
        if not (rec.count(b"\n") == 4 and rec.startswith(b"@SYN.%d " % (rid + 1))):
            raise SystemExit("record %d: seek returned %r" % (rid, rec[:40]))
        row = {"record": rid, "frac": frac, "bytes": len(rec), "total_ms": round(best, 3)}
        log(json.dumps(row))
        rec_rows.append(row)
    small = [r["total_ms"] for r in rows if r["len"] == 16384]
    return {
        "metric": "range seek latency, 16 KiB (device-resident, FASTQ-like)",
        "value": round(float(np.median(small)), 3), "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": 0,
        "ms_per_step": None, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "u8", "data": "synthetic",
        "config": {"workload": "FASTQ-like reads %d B, 12/16/24/32, 64 KiB blocks%s; best of %d seeks per point"
                               % (n, ", encoded in %d MiB segments" % (seg >> 20) if seg else "", args.steps)},
        "rows": rows, "record_seek": rec_rows,
    }


# distance classes named in Sec. 4.2 (d < 128, < 16384, < 2 Mi, else)
PAPER_BANDS = (128, 16384, 2097152)


def run_ablate(args, torch, lz):
    """Threshold and distance-band variants and schedule mechanisms on the
    FASTQ-like workload: the tuple the paper rejects (16/24/32/48), the paper's
    own distance bands with both headline tuples, the encoder's depth cap
    (6/8/10/12 at 64, 12/16/24/32 at 16 and 12), and, on 12/16/24/32, the
    decode without the one-workgroup tail, with G = 32, with schedule 0, and
    with the depth passes held to 6, 4 and 3 resident workgroups per CU (of
    8; the occupancy control of Sec. 3.3)."""
    import synth
    dev = torch.device("cuda:0")
    x = synth.fastq(args.size, seed=3)
    n = int(x.size)
    xt = torch.from_numpy(x).to(dev)
    rows = []
    variants = [("6/8/10/12", lz.BASE_THR, lz.BOUNDS_CFG, "cfg", 0),
                ("12/16/24/32", lz.TUNED_THR, lz.BOUNDS_CFG, "cfg", 0),
                ("16/24/32/48", (16, 24, 32, 48), lz.BOUNDS_CFG, "cfg", 0),
                ("6/8/10/12", lz.BASE_THR, PAPER_BANDS, "paper", 0),
                ("12/16/24/32", lz.TUNED_THR, PAPER_BANDS, "paper", 0),
                ("6/8/10/12", lz.BASE_THR, lz.BOUNDS_CFG, "cfg", 64),
                ("12/16/24/32", lz.TUNED_THR, lz.BOUNDS_CFG, "cfg", 16),
                ("12/16/24/32", lz.TUNED_THR, lz.BOUNDS_CFG, "cfg", 12)]
    tuned_gbps = None
    for name, thr, bounds, bname, cap in variants:
        log("encoding %s, %s bands, depth cap %d" % (name, bname, cap))
        arc = lz.encode(x, args.log2_bs, thr, bounds, max_chain=args.max_chain, depth_passes=args.depth_passes,
                        depth_cap=cap)
        info = lz.archive_info(arc)
        ent, _ = lz.entropy_size(arc)
        da = lz.DeviceArchive(arc, device=dev)
        out = torch.empty(n, dtype=torch.uint8, device=dev)
        mechs = [("G64 U2 schedule 1", 64, 2, 1, 0, 0)]
        if name == "12/16/24/32" and bname == "cfg" and not cap:
            mechs += [("no tail", 64, 2, 1, lz.TAIL_OFF, 0), ("G32", 32, 2, 1, 0, 0), ("schedule 0", 64, 2, 0, 0, 0)]
            mechs += [("occupancy %d of 8" % k, 64, 2, 1, 0, k) for k in (6, 4, 3)]
        for mname, G, U, S, T, O in mechs:
            da.decode(out, G=G, unroll=U, schedule=S, tail=T, occupancy=O)
            torch.cuda.synchronize()
            if not bool(torch.equal(out, xt)):
                raise SystemExit("ablation %s %s %s: decode differs from the input" % (name, bname, mname))
            steps = max(3, args.steps // (4 if S == 0 else 1))
            st = torch.cuda.current_stream()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            for _ in range(steps):
                da.decode_async(out, G=G, unroll=U, schedule=S, tail=T, occupancy=O)
            e1.record(st)
            e1.synchronize()
            da.check()
            ms = e0.elapsed_time(e1) / steps
            row = {"thr": name, "bands": bname, "depth_cap": cap, "mechanism": mname, "ms": round(ms, 4),
                   "gbps": round(n / ms / 1e6, 2), "depths": da.levels, "ratio_raw": round(n / arc.size, 4),
                   "ratio_entropy": round(n / ent, 4), "mean_match": round(info["mean_match"], 2),
                   "coverage": round(info["coverage"], 4)}
            log(json.dumps(row))
            rows.append(row)
            if name == "12/16/24/32" and bname == "cfg" and not cap and mname.startswith("G64"):
                tuned_gbps = row["gbps"]
        da.close()
        del out
        torch.cuda.empty_cache()
    rows += ablate_streams(args, torch, lz, x, xt)
    rows += ablate_source_order(args, torch, lz)
    return {
        "metric": "decode GB/s and ratio under threshold, band and schedule variants (FASTQ-like)",
        "value": tuned_gbps, "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u8", "data": "synthetic",
        "config": {"workload": "FASTQ-like reads %d B, 64 KiB blocks; bands cfg = 4 Ki/64 Ki/1 Mi, "
                               "paper = 128/16 Ki/2 Mi" % n},
        "rows": rows,
    }


def ablate_streams(args, torch, lz, x, xt):
    """Two concurrent decode streams (Sec. 3.3, last control): the tuned
    archive opened twice and decoded into two outputs on two streams at once,
    against one stream alone; aggregate output GB/s of each."""
    dev = torch.device("cuda:0")
    n = int(x.size)
    arc = lz.encode(x, args.log2_bs, lz.TUNED_THR, lz.BOUNDS_CFG, max_chain=args.max_chain,
                    depth_passes=args.depth_passes)
    das = [lz.DeviceArchive(arc, device=dev) for _ in range(2)]
    outs = [torch.empty(n, dtype=torch.uint8, device=dev) for _ in range(2)]
    sts = [torch.cuda.Stream() for _ in range(2)]
    for d, o, st in zip(das, outs, sts):
        d.decode(o, stream=st)
    torch.cuda.synchronize()
    steps = max(args.steps, 5)
    rows = []
    for k in (1, 2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            for d, o, st in list(zip(das, outs, sts))[:k]:
                d.decode_async(o, stream=st)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        for d, o, st in list(zip(das, outs, sts))[:k]:
            d.check(stream=st)
            if not bool(torch.equal(o, xt)):
                raise SystemExit("concurrent decode on %d streams differs from the input" % k)
        row = {"thr": "12/16/24/32", "bands": "cfg", "mechanism": "%d concurrent stream%s" % (k, "s" * (k > 1)),
               "ms_per_round": round(wall / steps * 1e3, 4), "aggregate_gbps": round(k * n * steps / wall / 1e9, 2)}
        log(json.dumps(row))
        rows.append(row)
    rows[-1]["vs_one_stream"] = round(rows[-1]["aggregate_gbps"] / rows[0]["aggregate_gbps"], 3)
    for d in das:
        d.close()
    del outs
    torch.cuda.empty_cache()
    return rows


def ablate_source_order(args, torch, lz, m=256, n=1 << 28):
    """Sorted against scattered source addresses (Sec. 3.3, third control) on
    the pure-copy path: the generated stream of mean match length m with its
    sources as generated (uniform over the output, scattered) and the same
    tokens with the sources sorted into increasing order, each copied from a
    reference buffer; every output checked against a plain PyTorch gather."""
    import synth
    dev = torch.device("cuda:0")
    ll, ml, sr, lit = synth.geo_tokens(n, m, seed=2 + 3)
    llv = np.asarray(ll, dtype=np.int64)
    mlv = np.asarray(ml, dtype=np.int64)
    mstart = np.concatenate([[0], np.cumsum(llv + mlv)[:-1]]) + llv
    dst = (mstart - llv).astype(np.uint64)
    loff = np.concatenate([[0], np.cumsum(llv)[:-1]]).astype(np.uint64)
    g = lambda a, dt: torch.from_numpy(np.ascontiguousarray(np.asarray(a).astype(dt))).to(dev)
    ref = torch.randint(0, 256, (n,), dtype=torch.uint8, device=dev)
    tlit = g(lit, np.uint8)
    us = g(copy_units(llv + mlv, 64, 2048), np.uint64)
    out = torch.empty(n, dtype=torch.uint8, device=dev)
    # the bytes each match must copy, for the check: output position -> reference position
    pos = torch.arange(n, device=dev, dtype=torch.int64)
    tok_of = torch.from_numpy(np.repeat(np.arange(llv.size), llv + mlv)).to(dev)
    rows = []
    srcs = {"scattered (as generated)": np.asarray(sr, dtype=np.int64),
            "sorted (increasing)": np.sort(np.asarray(sr, dtype=np.int64))}
    tdst, tlo, tll, tml = g(dst, np.uint64), g(loff, np.uint64), g(llv, np.uint32), g(mlv, np.uint32)
    for label, s in srcs.items():
        s = np.where(mlv > 0, s, 0)
        tsrc = g(s, np.uint64)
        pc = lz.PureCopy(tdst, tlo, tll, tsrc, tml, us, tlit, ref, out)
        pc.run(G=64, unroll=args.unroll)
        torch.cuda.synchronize()
        t_ms = torch.from_numpy(mstart).to(dev)[tok_of]
        in_match = pos >= t_ms
        want_ref = ref[(torch.from_numpy(s).to(dev)[tok_of] + (pos - t_ms)).clamp(0, n - 1)]
        want_lit = tlit[(torch.from_numpy(loff.astype(np.int64)).to(dev)[tok_of]
                         + (pos - torch.from_numpy(dst.astype(np.int64)).to(dev)[tok_of])).clamp(0, tlit.numel() - 1)]
        want = torch.where(in_match, want_ref, want_lit)
        if not bool(torch.equal(out, want)):
            raise SystemExit("pure copy with %s sources differs from the gather" % label)
        del want, want_ref, want_lit, in_match, t_ms
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(args.steps):
            pc.run(G=64, unroll=args.unroll)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / args.steps
        row = {"mechanism": "pure copy, %s sources" % label, "m": m, "n_bytes": n, "ms": round(ms, 4),
               "gbps": round(n / ms / 1e6, 2)}
        log(json.dumps(row))
        rows.append(row)
    rows[-1]["vs_scattered"] = round(rows[-1]["gbps"] / rows[0]["gbps"], 3)
    del out, ref, pos, tok_of
    torch.cuda.empty_cache()
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="fastq", choices=["fastq", "sweep", "batch", "serve", "ablate", "seek"])
    ap.add_argument("--count", type=int, default=4096, help="batch: archives")
    ap.add_argument("--requests", type=int, default=300, help="serve: requests")
    ap.add_argument("--capacity", default="0.5,0.8,0.95",
                    help="serve: offered rates as fractions of the saturated capacity (comma list)")
    ap.add_argument("--load", default="", help="serve: offered rate / one-at-a-time rate (comma list)")
    ap.add_argument("--arena", type=int, default=4096, help="serve: arena MiB")
    ap.add_argument("--slots", type=int, default=64, help="serve: request slots")
    ap.add_argument("--segment-mib", dest="segment_mib", type=int, default=-1,
                    help="serve/seek: encode in segments of this many MiB (serve default: 1024 above 3 GiB, else "
                         "none; seek default: none)")
    ap.add_argument("--size", type=int, default=1 << 30)
    ap.add_argument("--log2-bs", dest="log2_bs", type=int, default=16)
    ap.add_argument("--G", type=int, default=64)
    ap.add_argument("--unroll", type=int, default=2)
    ap.add_argument("--schedule", type=int, default=1)
    ap.add_argument("--max-chain", dest="max_chain", type=int, default=32)
    ap.add_argument("--depth-passes", dest="depth_passes", type=int, default=1,
                    help="encoder: depth-aware tie-break passes (0 = nearest source on ties)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-sweep-points", action="store_true",
                    help="fastq: skip the generated-stream points at mean match length 256 and 1024")
    ap.add_argument("--profile-run", action="store_true",
                    help="decode the 12/16/24/32 archive `steps` times plus a calibration kernel (counter runs)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the traffic summary from the counter CSVs of two --profile-run runs")
    ap.add_argument("--command", default="", help="with --traffic-from: the profiling command, recorded")
    args = ap.parse_args()
    if args.traffic_from:
        n = len(__import__("synth").fastq(args.size, seed=3))
        print(json.dumps(traffic_from_counters(args.traffic_from[0], args.traffic_from[1], args.steps, n,
                                               args.command, args.depth_passes)))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only; multi-GPU runs are not part of this build", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2607_18541_amd import lz
    if not torch.cuda.is_available():
        print("no GPU", file=sys.stderr)
        sys.exit(1)
    lz.lib()
    if args.profile_run:
        line = run_profile(args, torch, lz)
    elif args.workload == "sweep":
        if args.size == 1 << 30:
            args.size = 1 << 28
        line = run_sweep(args, torch, lz)
    elif args.workload == "batch":
        line = run_batch(args, torch, lz)
    elif args.workload == "serve":
        line = run_serve(args, torch, lz)
    elif args.workload == "ablate":
        line = run_ablate(args, torch, lz)
    elif args.workload == "seek":
        line = run_seek(args, torch, lz)
    else:
        line = run_fastq(args, torch, lz)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
