#!/usr/bin/env python3
"""Benchmark of the image-source RIR path on one MI355X.

One step = one batched launch over the 1024-room workload (seeded shoebox rooms
3-10 x 3-8 x 2.5-4 m, RT60 U[0.2, 0.8] s with Sabine reflection coefficients,
8-microphone 5 cm circular arrays, 16 kHz, RIR length 0.8 RT60 fs, 81-tap
Hann-windowed sinc): enumeration, FP64 delay split, tap evaluation and
accumulation, RIR store.  Inputs (the room table) are host arrays, as the API
takes them; outputs stay in HBM.

Printed: one JSON line with taps/s (value), RIRs/s batched and plain (one
launch per room), single-RIR latency percentiles, the roofline of the segment
kernel and the FP64 oracle's rate on the host cores (bounded sample).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "image-source taps/s + RIRs/s (batched vs plain, same GPU); p50/p99 RIR latency"
FLOPS_PER_TAP = 12          # nominal algorithmic flops per tap
FP32_VECTOR_PEAK_TFLOPS = 157.3


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("ism_kernels.hip", "ism_internal.h"):
        with open(os.path.join(ROOT, "paper_2104_13347_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(taps_per_launch):
    """HBM bytes per launch from the committed counter summary, if it was taken on the current
    kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "ism_segments_c1_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(batch, budget_s=12.0):
    import oracle
    nthreads = os.cpu_count() or 1
    R = len(batch["rir_len"])
    rng = np.random.default_rng(99)
    order = rng.permutation(R)
    taps = 0
    rirs = 0
    t0 = time.perf_counter()
    used = 0
    for i in range(0, R, 4):
        rooms = order[i:i + 4]
        lst = [(int(r), m) for r in rooms for m in range(int(batch["n_mics"][r]))]
        _, t = oracle.rir_list(batch, lst, nthreads=nthreads)
        taps += t
        rirs += len(lst)
        used += len(rooms)
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": taps / dt, "unit": "taps/s", "cores": nthreads, "kind": "oracle",
            "rirs_per_s": rirs / dt,
            "sample": f"{used} random rooms of the 1024-room batch, all 8 mics ({rirs} RIRs, {taps} taps), "
                      f"FP64 oracle, {nthreads} threads over RIRs, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--rooms", type=int, default=1024)
    ap.add_argument("--precision", type=int, default=0)
    ap.add_argument("--seg-len", type=int, default=0)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--latency-reps", type=int, default=200)
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="run only a plain device copy of this many bytes (HBM counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the path shards by room with no "
              "exchange, see DESIGN.md", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2104_13347_amd import ism, scenes

    assert torch.cuda.is_available(), "needs a GPU"
    dev = torch.device("cuda:0")
    batch = scenes.c1(n_rooms=args.rooms)
    rooms = ism.rooms_array(batch)
    n_rirs = int(batch["n_mics"].sum())
    H = ism.Handle()
    if args.seg_len:
        H.set_tuning(seg_len=args.seg_len)
    out = torch.empty(int(batch["out_size"]), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        H.rir_batch(batch, precision=args.precision, out=out, rooms=rooms)
    torch.cuda.synchronize()
    counts = H.last_counts()

    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        evs[i][0].record(stream)
        H.rir_batch(batch, precision=args.precision, out=out, rooms=rooms)
        evs[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launch_ms = [a.elapsed_time(b) for a, b in evs]
    ms_per_step = wall * 1e3 / args.steps
    taps = counts["taps"]
    value = taps / (ms_per_step / 1e3)
    rirs_batched = n_rirs / (ms_per_step / 1e3)
    k_ms = float(np.mean(launch_ms))

    res = {"metric": METRIC, "value": value, "unit": "taps/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "c1: 1024 seeded shoebox rooms x 8 mics, 16 kHz, RIR 0.8*RT60*fs, "
                                  "81-tap Hann-windowed sinc, time-bounded image sets",
                      "rooms": args.rooms, "rirs": n_rirs, "taps_per_step": taps,
                      "records_per_step": counts["records"], "images_tested_per_step": counts["images"],
                      "precision": ["fp32", "fp16_lut", "fp32_split", "fp32_atomic"][args.precision],
                      "tuning": H.get_tuning()},
           "rirs_per_s_batched": rirs_batched}

    # roofline of the segment kernel (the launch is one graph: upload + prologue + segments)
    achieved = FLOPS_PER_TAP * taps / (k_ms / 1e3) / 1e12
    traffic = measured_traffic(taps)
    res["roofline"] = {"bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFLOPS,
                       "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK_TFLOPS, "traffic": traffic,
                       "kernel": "ism_segments", "launch_ms": k_ms,
                       "flops_per_tap": FLOPS_PER_TAP, "taps_per_launch": taps}

    # plain: the same kernels launched once per room, host loop, one stream
    if not args.no_plain:
        M = int(batch["n_mics"][0])
        mics_all = batch["mics"]
        for r in range(min(8, args.rooms)):   # warm-up
            o, L, mo = int(batch["out_offset"][r]), int(batch["rir_len"][r]), int(batch["mic_offset"][r])
            H.rir(batch["L"][r], batch["beta"][r], batch["src"][r], mics_all[mo:mo + M], batch["fs"], batch["c"],
                  -1, L, batch["fd_taps"], out=out[o:o + M * L].view(M, L))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for r in range(args.rooms):
            o, L, mo = int(batch["out_offset"][r]), int(batch["rir_len"][r]), int(batch["mic_offset"][r])
            H.rir(batch["L"][r], batch["beta"][r], batch["src"][r], mics_all[mo:mo + M], batch["fs"], batch["c"],
                  -1, L, batch["fd_taps"], out=out[o:o + M * L].view(M, L))
        torch.cuda.synchronize()
        plain_s = time.perf_counter() - t0
        res["rirs_per_s_plain"] = n_rirs / plain_s
        res["taps_per_s_plain"] = taps / plain_s
        res["batched_vs_plain"] = rirs_batched / res["rirs_per_s_plain"]

    # single-RIR latency (the 5x4x3 m order-10 room, one mic, 4096 samples), launch to completion
    c0 = scenes.c0()
    lat = []
    o1 = torch.empty((1, 4096), dtype=torch.float32, device=dev)
    for i in range(args.latency_reps + 10 if args.latency_reps > 0 else 0):
        torch.cuda.synchronize()
        t = time.perf_counter()
        H.rir(c0["L"][0], c0["beta"][0], c0["src"][0], c0["mics"], c0["fs"], c0["c"], 10, 4096, 81, out=o1)
        torch.cuda.synchronize()
        if i >= 10:
            lat.append((time.perf_counter() - t) * 1e3)
    if lat:
        res["latency_ms_single_rir"] = {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                                        "workload": "5x4x3 m room, index-L1 order 10, 1 mic, 4096 samples"}
    H.close()

    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(batch)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
