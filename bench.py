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
# nominal algorithmic flops per tap of the rational tap form: subtract, reciprocal, two FMAs
# (4 flops), two multiplies, and 4 for an accurate (compensated) accumulation
FLOPS_PER_TAP = 12
FP32_VECTOR_PEAK_TFLOPS = 157.3
# what each precision mode computes in: FP64 geometry and delay split throughout; the default
# evaluates FP64 Chebyshev moments, sums them exactly in 64-bit integer bins and runs the filter on
# the matrix cores over FP16 pairs (hi*hi + hi*lo + lo*hi) with FP32 sums
DTYPES = ["f64+int64+f16pair-mfma", "f64+f16-lut+int64", "f32-split+int64+f16pair-mfma", "f64+f32-atomic",
          "f64+f32+int64"]


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("ism_kernels.hip", "ism_internal.h"):
        with open(os.path.join(ROOT, "paper_2104_13347_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def committed_counters(kernel):
    """The committed counter summary of `kernel` on the 1024-room batch, if it was taken on
    the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_c1_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d


def measured_traffic(kernel):
    """HBM bytes per launch from the committed counter summary, or None."""
    d = committed_counters(kernel)
    return d.get("hbm_bytes_per_launch") if d else None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def rir_errors(batch, gpu, ref, rirs):
    """max |gpu - oracle| / max |oracle| of each listed (room, mic) RIR (flat batch layout)."""
    errs = []
    for r, m in rirs:
        L = int(batch["rir_len"][r])
        o = int(batch["out_offset"][r]) + m * L
        g, f = gpu[o:o + L].astype(np.float64), ref[o:o + L]
        errs.append(float(np.abs(g - f).max() / max(np.abs(f).max(), 1e-300)))
    return np.array(errs)


def cpu_baseline(batch, gpu=None, budget_s=12.0, total_taps=None):
    """The FP64 oracle on the host cores (threads over RIRs) on a bounded random sample of the
    batch's rooms; with `gpu` (the batch's GPU output, host copy) the sample's RIRs are also
    compared with it, so the headline run carries its own error against the oracle."""
    import oracle
    nthreads = os.cpu_count() or 1
    R = len(batch["rir_len"])
    rng = np.random.default_rng(99)
    order = rng.permutation(R)
    ref = np.zeros(int(batch["out_size"]))
    taps = 0
    done = []
    t0 = time.perf_counter()
    used = 0
    for i in range(0, R, 4):
        rooms = order[i:i + 4]
        lst = [(int(r), m) for r in rooms for m in range(int(batch["n_mics"][r]))]
        _, t = oracle.rir_list(batch, lst, nthreads=nthreads, out=ref)
        taps += t
        done += lst
        used += len(rooms)
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    # single-core rate on the first two RIRs of the sample
    t1 = time.perf_counter()
    _, t_one = oracle.rir_list(batch, done[:2], nthreads=1)
    one_core = t_one / (time.perf_counter() - t1)
    res = {"value": taps / dt, "unit": "taps/s", "cores": nthreads, "kind": "oracle",
           "cpu_model": cpu_model(), "single_core_taps_per_s": one_core,
           "rirs_per_s": len(done) / dt,
           "sample": f"{used} random rooms of the 1024-room batch, all 8 mics ({len(done)} RIRs, {taps} taps), "
                     f"FP64 oracle, {nthreads} threads over RIRs, {dt:.1f} s"}
    if total_taps:
        res["full_batch_s_extrapolated"] = total_taps / res["value"]
    if gpu is not None:
        e = rir_errors(batch, gpu, ref, done)
        res["gpu_vs_oracle"] = {"rirs": len(done), "max_err_over_peak": float(e.max()),
                                "median_err_over_peak": float(np.median(e)), "bar": 1e-5}
    return res


def _time_it(torch, fn, reps=3):
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.median(ts))


def bench_c3(H, torch, with_errors=True):
    """64 rooms 20x15x8 m, 48 kHz, 72000 samples, 16 mics, 127 taps: throughput per precision mode,
    and each mode's error against the FP64 oracle on a sample of RIRs (every microphone of rooms
    0 and 37, computed once on the host cores)."""
    from paper_2104_13347_amd import ism, scenes
    b = scenes.c3()
    rooms = ism.rooms_array(b)
    out = torch.empty(int(b["out_size"]), dtype=torch.float32, device="cuda")
    res = {"workload": "64 rooms 20x15x8 m, per-wall beta U[0.85,0.95], 48 kHz, 72000 samples, 16 mics, 127 taps"}
    sample = [(r, m) for r in (0, 37) for m in range(16)]
    ref = None
    if with_errors:
        import oracle
        ref = np.zeros(int(b["out_size"]))
        t = time.perf_counter()
        _, otaps = oracle.rir_list(b, sample, out=ref)
        dt = time.perf_counter() - t
        res["error_sample"] = "all 16 mics of rooms 0 and 37 (32 RIRs), FP64 oracle"
        res["cpu_oracle_on_sample"] = {"taps_per_s": otaps / dt, "rirs_per_s": len(sample) / dt, "s": dt,
                                       "cores": os.cpu_count() or 1}
    bars = {"fp32": 1e-5, "fp32_direct": 1e-5, "fp16_lut": 2e-3, "fp32_split": None}
    for prec, name in [(ism.PREC_FP32, "fp32"), (ism.PREC_FP32_DIRECT, "fp32_direct"), (ism.PREC_FP16_LUT, "fp16_lut"),
                       (ism.PREC_FP32_SPLIT, "fp32_split")]:
        ms = _time_it(torch, lambda: H.rir_batch(b, precision=prec, out=out, rooms=rooms))
        taps = H.last_counts()["taps"]
        res[name] = {"ms": ms, "taps_per_s": taps / (ms / 1e3), "rirs_per_s": 64 * 16 / (ms / 1e3), "taps": taps}
        if ref is not None:
            e = rir_errors(b, out.cpu().numpy(), ref, sample)
            res[name]["max_err_over_peak"] = float(e.max())
            res[name]["median_err_over_peak"] = float(np.median(e))
            res[name]["bar"] = bars[name]
    return res


def bench_c0_replicated(H, torch, with_errors=True):
    """The single-RIR room (5 x 4 x 3 m, beta 0.7, index-L1 order 10, 4096 samples, 81 taps)
    as 4096 rooms of identical shape with sources moved by up to 0.25 m: the per-RIR work of
    the latency workload at a batch size that fills the chip.  Errors against the FP64 oracle
    on 8 of the rooms."""
    from paper_2104_13347_amd import ism, scenes
    b = scenes.c0_replicated()
    rooms = ism.rooms_array(b)
    out = torch.empty(int(b["out_size"]), dtype=torch.float32, device="cuda")
    ms = _time_it(torch, lambda: H.rir_batch(b, out=out, rooms=rooms), reps=5)
    taps = H.last_counts()["taps"]
    tf = taps * FLOPS_PER_TAP / (ms / 1e3) / 1e12
    res = {"workload": "4096 copies of the 5x4x3 m, beta 0.7, index-L1 order 10 room, 1 mic, 4096 samples, "
                       "81 taps, sources moved by U[-0.25, 0.25] m per axis",
           "ms": ms, "taps": taps, "taps_per_s": taps / (ms / 1e3), "rirs_per_s": 4096 / (ms / 1e3),
           "nominal_tflops": tf, "nominal_frac": tf / FP32_VECTOR_PEAK_TFLOPS,
           "note": "taps x 12 nominal flops of the direct method over the FP32 vector peak"}
    if with_errors:
        import oracle
        sample = [(r, 0) for r in range(0, 4096, 512)]
        ref = np.zeros(int(b["out_size"]))
        t = time.perf_counter()
        _, otaps = oracle.rir_list(b, sample, out=ref)
        dt = time.perf_counter() - t
        e = rir_errors(b, out.cpu().numpy(), ref, sample)
        res["gpu_vs_oracle"] = {"rirs": len(sample), "max_err_over_peak": float(e.max()),
                                "median_err_over_peak": float(np.median(e)), "bar": 1e-5}
        res["cpu_oracle_on_sample"] = {"taps_per_s": otaps / dt, "s": dt, "cores": os.cpu_count() or 1}
    del out
    return res


def bench_paper(H, torch):
    """The paper's room dataset: 7 x 10 x 3.7 m, RT 0.5 s, 48 000 torus source positions x the
    7-microphone array = 336 000 RIRs of 8000 samples (16 kHz), in one batched launch, with the
    paper's 7th-order Lagrange filter and with the 81-tap windowed sinc."""
    from paper_2104_13347_amd import ism, scenes
    b = scenes.paper_room1()
    rooms = ism.rooms_array(b)
    out = torch.empty(int(b["out_size"]), dtype=torch.float32, device="cuda")
    n_rirs = int(b["n_mics"].sum())
    res = {"workload": "paper room 1: 7x10x3.7 m, RT 0.5 s, 48000 sources x 7 mics = 336000 RIRs x 8000 "
                       "samples at 16 kHz", "rirs": n_rirs, "output_bytes": int(b["out_size"]) * 4}
    for taps, name in [(8, "lagrange_fd8"), (81, "sinc_fd81")]:
        b["fd_taps"] = taps
        ms = _time_it(torch, lambda: H.rir_batch(b, precision=ism.PREC_FP32, out=out, rooms=rooms), reps=2)
        cnt = H.last_counts()
        res[name] = {"ms": ms, "rirs_per_s": n_rirs / (ms / 1e3), "taps_per_s": cnt["taps"] / (ms / 1e3),
                     "records": cnt["records"], "taps": cnt["taps"]}
    del out
    torch.cuda.empty_cache()
    return res


def bench_c4(H, torch, with_errors=True, two_streams=True):
    """256 rooms (1024-room distribution, seed 2108), 8 mics: RIR batch on the GPU, then convolution
    with 1 s white-noise sources and sensor noise at SNR U[0,30] dB.  With errors: the noisy
    recordings of rooms 0, 128 and 255 against the FP64 oracle's convolution of the same GPU RIRs
    plus the oracle's own deviates for the same seed (relative RMS per room, both paths)."""
    from paper_2104_13347_amd import ism, scenes
    b = scenes.c4(with_z=False)
    rooms = ism.rooms_array(b)
    rirs = torch.empty(int(b["out_size"]), dtype=torch.float32, device="cuda")
    x = torch.from_numpy(b["x"]).cuda()
    y = torch.empty((256, 8, 16000), dtype=torch.float32, device="cuda")
    seed = b["noise_seed"]
    lens = b["rir_len"]
    offs = b["out_offset"]
    rir_ms = _time_it(torch, lambda: H.rir_batch(b, out=rirs, rooms=rooms))
    flops = 0.0
    for L in lens:   # algorithmic MACs: sum over n < 16000 of min(n + 1, L)
        L = int(L)
        flops += 2.0 * 8 * (L * 16000 - L * (L - 1) / 2.0)
    res = {"workload": "256 rooms x 8 mics, RIR 0.8*RT60*fs, 1 s N(0,1) source at 16 kHz, SNR U[0,30] dB, "
                       "sensor noise drawn on the device (Philox4x32-10 + Box-Muller)",
           "rir_batch_ms": rir_ms, "algorithmic_flops": flops}
    n_seq = 8   # throughput: per call within 8 back-to-back calls on one stream
    for mfma, name in [(True, "bf16_mfma"), (False, "fp32_direct")]:
        noisy = lambda: H.convolve_batch(rirs, offs, lens, 8, x, 16000, snr_db=b["snr_db"], noise_seed=seed,
                                         use_mfma=mfma, out=y)
        clean = lambda: H.convolve_batch(rirs, offs, lens, 8, x, 16000, use_mfma=mfma, out=y)
        ms = _time_it(torch, lambda: [noisy() for _ in range(n_seq)]) / n_seq
        ms_clean = _time_it(torch, lambda: [clean() for _ in range(n_seq)]) / n_seq
        tf = flops / (ms_clean / 1e3) / 1e12
        peak = 2500.0 if mfma else FP32_VECTOR_PEAK_TFLOPS
        # each kernel alone: HIP events the library records around its kernels (median of 5 calls)
        H.set_conv_timing(True)
        try:
            kt = []
            for _ in range(5):
                noisy()
                kt.append(H.conv_last_timing())
        finally:
            H.set_conv_timing(False)
        kpk, kcv, knz = (float(np.median([t[i] for t in kt])) for i in range(3))
        two = {}
        if mfma and two_streams:
            # calls alternating between two streams and two outputs: one call's noise pass and
            # the next call's pack run beside the other stream's convolution kernel
            ss, y2 = [torch.cuda.Stream(), torch.cuda.Stream()], [y, torch.empty_like(y)]

            def two_streams():
                cur = torch.cuda.current_stream()
                for s in ss:
                    s.wait_stream(cur)
                for i in range(n_two):
                    H.convolve_batch(rirs, offs, lens, 8, x, 16000, snr_db=b["snr_db"], noise_seed=seed,
                                     use_mfma=True, out=y2[i % 2], stream=ss[i % 2])
                for s in ss:
                    cur.wait_stream(s)
            n_two = 16
            ms2 = _time_it(torch, two_streams, reps=5) / n_two
            del y2
            two = {"ms_with_noise_two_streams": ms2, "timing_two_streams": f"per call, {n_two} calls in turn on two streams",
                   "path_frac_two_streams": flops / (ms2 / 1e3) / 1e12 / peak}
        res[name] = {"ms_with_noise": ms, "ms_convolution_only": ms_clean, "timing": f"per call, {n_seq} calls back to back",
                     "ms_single_call_with_noise": _time_it(torch, noisy), "tflops": tf,
                     "peak_tflops": peak, "frac": tf / peak,
                     "path_tflops": flops / (ms / 1e3) / 1e12, "path_frac": flops / (ms / 1e3) / 1e12 / peak,
                     "kernel_ms": {"pack": kpk, "convolution": kcv, "noise": knz,
                                   "timing": "HIP events around each kernel, median of 5 calls"},
                     "kernel_tflops": flops / (kcv / 1e3) / 1e12, "kernel_frac": flops / (kcv / 1e3) / 1e12 / peak,
                     **two}
        if with_errors:
            import oracle
            from oracle import noise
            H.convolve_batch(rirs, offs, lens, 8, x, 16000, snr_db=b["snr_db"], noise_seed=seed, use_mfma=mfma, out=y)
            got, hr = y.cpu().numpy(), rirs.cpu().numpy()
            errs = []
            for r in (0, 128, 255):
                L = int(lens[r])
                h = hr[offs[r]:offs[r] + 8 * L].reshape(8, L).astype(np.float64)
                ref = oracle.conv_room(h, b["x"][r].astype(np.float64), 16000, snr_db=float(b["snr_db"][r]),
                                       z=noise.deviates(seed, r, 8, 16000))
                errs.append(float(np.sqrt(np.mean((got[r] - ref) ** 2) / np.mean(ref ** 2))))
            res[name]["rel_rms_err"] = {"rooms": [0, 128, 255], "values": errs,
                                        "bar": 1e-2 if mfma else None}
    res["noise_pass_ms"] = res["bf16_mfma"]["ms_with_noise"] - res["bf16_mfma"]["ms_convolution_only"]

    def pipeline():   # RIRs, convolution and device-drawn noise
        H.rir_batch(b, out=rirs, rooms=rooms)
        H.convolve_batch(rirs, offs, lens, 8, x, 16000, snr_db=b["snr_db"], noise_seed=seed, out=y)
    res["pipeline_ms"] = _time_it(torch, pipeline)
    return res


def bench_beamlearning(H, torch):
    """BeamLearning forward pass (section II.B) over 3600 frames of 7 x 1024 samples, the size of
    the paper's 3600-localisation test set, cut on the device from the recordings of the
    convolution stage (256 rooms, 8 mics, 1 s at 16 kHz; 15 frames per room, 7 of the 8
    channels) through per-frame offsets.  Weights drawn as the paper initialises them.  The
    paper times its inference one frame at a time, so the one-frame latency is reported too."""
    from paper_2104_13347_amd import beamlearning as blm, bl_data, ism, scenes
    b = scenes.c4(with_z=False)
    rooms = ism.rooms_array(b)
    rirs = torch.empty(int(b["out_size"]), dtype=torch.float32, device="cuda")
    H.rir_batch(b, out=rirs, rooms=rooms)
    y = H.convolve_batch(rirs, b["out_offset"], b["rir_len"], 8, torch.from_numpy(b["x"]).cuda(), 16000,
                         snr_db=b["snr_db"], noise_seed=b["noise_seed"])
    B, NT, CIN = 3600, 1024, 7
    idx = np.arange(B)
    offs = torch.from_numpy((idx // 15) * 8 * 16000 + (idx % 15) * NT).to(torch.int64).cuda()
    model = blm.Model(H, bl_data.flatten(bl_data.make_params(2104), CIN, 2), c_in=CIN, n_out=2)
    ws = torch.empty(blm.workspace_bytes(B, NT), dtype=torch.uint8, device="cuda")
    out = torch.empty((B, 2), dtype=torch.float32, device="cuda")
    run = lambda: model.forward(y, n_t=NT, batch=B, offsets=offs, ch_stride=16000, workspace=ws,
                                features=False, out=out)
    ms = _time_it(torch, run, reps=5)
    xs = torch.from_numpy(b["x"]).cuda()

    def pipeline():  # RIRs of the 256 rooms, their recordings, then the network on 3600 frames
        H.rir_batch(b, out=rirs, rooms=rooms)
        H.convolve_batch(rirs, b["out_offset"], b["rir_len"], 8, xs, 16000, snr_db=b["snr_db"],
                         noise_seed=b["noise_seed"], out=y)
        run()
    pipe_ms = _time_it(torch, pipeline, reps=3)
    ws1 = torch.empty(blm.workspace_bytes(1, NT), dtype=torch.uint8, device="cuda")
    out1 = torch.empty((1, 2), dtype=torch.float32, device="cuda")
    one = lambda: model.forward(y, n_t=NT, batch=1, offsets=offs[:1], ch_stride=16000, workspace=ws1,
                                features=False, out=out1)
    lat = [_time_it(torch, one, reps=1) for _ in range(30)]
    # small batches (16- and 32-row tiles below 256 workgroups per layer): p50 per call
    ws16 = torch.empty(blm.workspace_bytes(16, NT), dtype=torch.uint8, device="cuda")
    out16 = torch.empty((16, 2), dtype=torch.float32, device="cuda")
    small = {}
    for nb in (2, 4, 8, 16):
        call = lambda: model.forward(y, n_t=NT, batch=nb, offsets=offs[:nb], ch_stride=16000, workspace=ws16,
                                     features=False, out=out16[:nb])
        small[str(nb)] = float(np.median([_time_it(torch, call, reps=1) for _ in range(15)]))
    # algorithmic HBM bytes per frame: layer 0 reads the frame and writes a_0; layer 1 reads
    # a_0 and writes x_1, a_1; layers 2..17 read a, x and write x, a; the pseudo-energy reads
    # a_17 and x_17 on the valid samples
    m = NT * 128 * 4
    per_frame = CIN * NT * 4 + m + 3 * m + 16 * 4 * m + 2 * (NT - 2 * 189) * 128 * 4
    gbs = B * per_frame / (ms / 1e3) / 1e9
    # the method's own arithmetic per frame (section II.B): per layer a depthwise convolution
    # (3 taps, channel multiplier 4) and a pointwise one onto 128 channels, 2 flops per MAC
    flops_frame = 2.0 * NT * (3 * 4 * CIN + 4 * CIN * 128) + 17 * 2.0 * NT * (3 * 4 * 128 + 4 * 128 * 128)
    tfl = B * flops_frame / (ms / 1e3) / 1e12
    model.close()
    return {"workload": "3600 frames x 7 ch x 1024 samples cut from 256 rooms x 8 mics x 1 s recordings; "
                        "18 filterbank layers + pseudo-energy + head, paper-initialised weights",
            "ms": ms, "frames_per_s": B / (ms / 1e3), "us_per_frame": ms * 1e3 / B,
            "pipeline_ms": pipe_ms,  # RIRs (256 rooms x 8 mics) + convolution + forward pass
            "batch1_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
            "small_batch_p50_ms": small,
            "paper_gtx1080ti_batch1_ms": 16.2e3 / 3600,
            "algorithmic_flops_per_frame": flops_frame,
            "roofline": {"bound": "mfma", "achieved": tfl, "peak": 2500.0, "unit": "TFLOP/s", "frac": tfl / 2500.0,
                         "note": "the method's depthwise + pointwise flops per frame over the dense FP16 peak; the "
                                 "kernels run the folded layers as FP16 pairs (three products per step), so their "
                                 "own ceiling for this arithmetic is a third of that peak"},
            "hbm_structure": {"bytes_per_frame": per_frame, "achieved_gbs": gbs, "peak_gbs": 8000.0,
                              "frac": gbs / 8000.0,
                              "note": "reads and writes of the layer-by-layer maps this structure needs "
                                      "(the frame itself is 28.7 KB)"}}


def cpu_baseline_beamlearning(n_frames=2):
    """The FP64 BeamLearning oracle on a bounded sample: n_frames frames of 7 x 1024."""
    from oracle import beamlearning as ref
    from paper_2104_13347_amd import bl_data
    p = bl_data.make_params(2104)
    x = bl_data.frames(7, n_frames)
    t = time.perf_counter()
    ref.forward(x, p)
    s = (time.perf_counter() - t) / n_frames
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"] or [1])
    except Exception:
        cores = 1
    return {"value": 1.0 / s, "unit": "frames/s", "cores": cores, "kind": "oracle",
            "sample": f"{n_frames} frames of 7 x 1024, numpy FP64 (BLAS threads for the pointwise products)"}


def bench_rt_fit(H, torch):
    """Uniform-absorption fit (section III.A: homogeneous walls with a simulated reverberation
    time of 0.5 s) for the paper's two simulated rooms, then each room's 336 000-RIR dataset with
    the fitted walls.  Room-level fit: the mean T30 of the RIRs from the first 8 torus sources of
    the room's dataset to the 7 array microphones (56 RIRs of 16 000 samples per step, Lagrange
    filter, 16 kHz, 30 bisection steps).  The single-pair fit (array centre, one source 2 m away)
    and Sabine's coefficient are given for comparison."""
    from paper_2104_13347_amd import ism, scenes
    res = {"workload": "paper rooms 7x10x3.7 m and 5x5x4 m, target T30 0.5 s; room-level fit on the mean T30 of "
                       "8 torus sources x 7 mics (16 kHz, 16000 samples, fd_taps 8, 30 bisection steps), then the "
                       "room's 48000-source x 7-mic dataset (8000 samples) with the fitted beta"}
    rooms = {"room1_7x10x3.7": (scenes.paper_room1, [7.0, 10.0, 3.7], [4.0, 6.0, 1.5], [6.0, 6.0, 1.5]),
             "room2_5x5x4": (scenes.paper_room2, [5.0, 5.0, 4.0], [2.5, 2.5, 1.5], [4.5, 2.5, 1.5])}
    for name, (scene, L, mic, src) in rooms.items():
        probe = scene(n_sources=8)
        srcs, mics = probe["src"], probe["mics"][:7]
        H.fit_beta_mean(L, srcs, mics, 16000.0, 343.0, 8, 0.5, 16000, iters=30)   # warm-up, same steps
        torch.cuda.synchronize()
        t = time.perf_counter()
        beta, rt = H.fit_beta_mean(L, srcs, mics, 16000.0, 343.0, 8, 0.5, 16000, iters=30)
        fit_ms = (time.perf_counter() - t) * 1e3
        b1, rt1 = H.fit_beta(L, src, mic, 16000.0, 343.0, 8, 0.5, 16000, iters=30)
        b = scene(beta=beta)
        rooms_t = ism.rooms_array(b)
        out = torch.empty(int(b["out_size"]), dtype=torch.float32, device="cuda")
        ms = _time_it(torch, lambda: H.rir_batch(b, out=out, rooms=rooms_t), reps=2)
        cnt = H.last_counts()
        n_rirs = int(b["n_mics"].sum())
        res[name] = {"beta_room_fit": beta, "mean_t30_s": rt, "room_fit_ms": fit_ms,
                     "beta_single_pair_fit": b1, "single_pair_t30_s": rt1,
                     "beta_sabine": float(scene(n_sources=1)["beta"][0][0]),
                     "dataset": {"rirs": n_rirs, "ms": ms, "rirs_per_s": n_rirs / (ms / 1e3),
                                 "taps_per_s": cnt["taps"] / (ms / 1e3), "taps": cnt["taps"],
                                 "output_bytes": int(b["out_size"]) * 4}}
        del out
        torch.cuda.empty_cache()
    return res


def cpu_oracle_c2(b, total_taps, budget_s=8.0, max_requests=256):
    """The FP64 oracle on a seeded subset of the serving requests (at most 256, bounded to
    about budget_s), threads over each request's RIRs; its rate extrapolated to every
    request's taps (the device's exact count)."""
    import oracle
    from paper_2104_13347_amd import scenes
    nthreads = os.cpu_count() or 1
    idx = np.random.default_rng(2106).choice(len(b["rir_len"]), size=min(max_requests, len(b["rir_len"])),
                                             replace=False)
    sub = scenes.subset(b, idx)
    ref = np.zeros(int(sub["out_size"]))
    taps, done = 0, 0
    t0 = time.perf_counter()
    i = 0
    while i < len(idx):   # requests in groups of at least one RIR per thread
        lst = []
        while i < len(idx) and len(lst) < nthreads:
            lst += [(i, m) for m in range(int(sub["n_mics"][i]))]
            i += 1
        _, t = oracle.rir_list(sub, lst, nthreads=nthreads, out=ref)
        taps += t
        done = i
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    return {"requests": done, "taps": taps, "s": dt, "taps_per_s": taps / dt, "requests_per_s": done / dt,
            "cores": nthreads, "kind": "oracle",
            "sample": f"{done} of a seeded subset of {len(idx)} requests, FP64 oracle, {nthreads} threads over RIRs",
            "all_requests_s_extrapolated": total_taps / (taps / dt) if total_taps else None}


def bench_c2(torch, n_requests, batched_taps_per_s=None, with_oracle=False):
    """Serving: Poisson arrivals of single-room requests (RT60 U[0.1,1.0] s, RIR RT60*fs, M in
    {4,8,16,32}).  A saturated run (all requests at t=0) on the 8 GB engine gives the sustainable
    rate; arrivals at 0.7 of it then run three times on each HBM budget (8 GB, 1 GB, and 32 MB,
    where admission binds), giving p50/p99 latency per replay and served taps/s (exact device
    counts).  The budget covers the output pool and every lane's staging slots."""
    from paper_2104_13347_amd import ism, scenes
    reqs, gaps, meta = scenes.c2(n_requests=n_requests)
    b = scenes.pack(reqs, meta["fs"], meta["c"], meta["fd_taps"], meta["order_mode"], "c2")
    n_rirs = int(b["n_mics"].sum())
    res = {"workload": f"{n_requests} requests, Poisson arrivals, RT60 U[0.1,1.0] s, M in {{4,8,16,32}}, 16 kHz",
           "lanes": 4, "max_batch_rooms": 64, "replays_per_budget": 3}
    lam = total_taps = None
    for name, budget in [("budget_8GiB", 8 << 30), ("budget_1GiB", 1 << 30), ("budget_32MiB", 32 << 20)]:
        S = ism.Server(n_lanes=4, hbm_budget_bytes=budget, max_batch_rooms=64)
        try:
            c0 = S.counters()
            lat0, wall0 = S.replay(b, np.zeros(n_requests))
            c1 = S.counters()
            entry = {"saturated": {"requests_per_s": n_requests / wall0, "rirs_per_s": n_rirs / wall0,
                                   "taps_per_s": (c1["taps_done"] - c0["taps_done"]) / wall0, "wall_s": wall0}}
            if total_taps is None:
                total_taps = c1["taps_done"] - c0["taps_done"]
            if lam is None:
                lam = 0.7 * n_requests / wall0
            reps = []
            for _ in range(3):
                a = S.counters()
                lat, wall = S.replay(b, np.cumsum(gaps) / lam)
                z = S.counters()
                reps.append({"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                             "rirs_per_s": n_rirs / wall, "taps_per_s": (z["taps_done"] - a["taps_done"]) / wall,
                             "wall_s": wall, "admission_stalls": z["admission_stalls"] - a["admission_stalls"]})
            p99 = [r["p99_ms"] for r in reps]
            st, cn = S.stats(), S.counters()
            entry["poisson"] = {
                "lambda_per_s": lam, "replays": reps,
                "p50_ms_median": float(np.median([r["p50_ms"] for r in reps])),
                "p99_ms_median": float(np.median(p99)), "p99_ms_range": [float(min(p99)), float(max(p99))],
                "served_taps_per_s_median": float(np.median([r["taps_per_s"] for r in reps]))}
            if batched_taps_per_s:
                entry["poisson"]["served_vs_batched_taps"] = entry["poisson"]["served_taps_per_s_median"] / \
                    batched_taps_per_s
                entry["saturated"]["served_vs_batched_taps"] = entry["saturated"]["taps_per_s"] / batched_taps_per_s
            entry["memory"] = {"budget_bytes": cn["budget_bytes"], "pool_bytes": cn["pool_bytes"],
                               "staging_bytes": cn["staging_bytes"], "pool_peak_bytes": cn["pool_peak_bytes"],
                               "admission_stalls_total": cn["admission_stalls"]}
            entry["max_concurrent_batches"] = st["max_concurrent_batches"]
            entry["batches"] = st["batches"]
            res[name] = entry
        finally:
            S.close()
    if with_oracle:
        res["cpu_oracle"] = cpu_oracle_c2(b, total_taps)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--rooms", type=int, default=1024)
    ap.add_argument("--precision", type=int, default=0)
    ap.add_argument("--seg-len", type=int, default=0, help="fixed segment length (no autotuning)")
    ap.add_argument("--no-autotune", action="store_true", help="launch with the default tuning")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ablation", action="store_true",
                    help="skip the per-tap (direct) evaluation of the same batch")
    ap.add_argument("--latency-reps", type=int, default=200)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the serving, precision and convolution sections")
    ap.add_argument("--extras", default="c0x,c3,c4,paper,c2,beamlearning,rtfit",
                    help="comma list of extra sections to run: c0x (the single-RIR room as 4096 rooms), "
                         "c3 precision, c4 convolution, paper (the "
                         "paper's 336 000-RIR room dataset), c2 serving, beamlearning (the paper's network "
                         "on frames of the convolution stage), rtfit (uniform-absorption fit for a target T30)")
    ap.add_argument("--serve-requests", type=int, default=20000)
    ap.add_argument("--no-two-streams", action="store_true",
                    help="leave out the convolution calls on two streams (their kernels overlap)")
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
              "exchange between GPUs", file=sys.stderr)
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
    tune_s = None
    if not args.seg_len and not args.no_autotune:
        # one-time set-up before the warm-up: the batch's shape bucket is tuned on its first launch
        H.set_autotune(True)
        t = time.perf_counter()
        H.rir_batch(batch, precision=args.precision, out=out, rooms=rooms)
        torch.cuda.synchronize()
        tune_s = time.perf_counter() - t

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
    gpu_out = out.cpu().numpy() if not args.no_cpu_baseline else None   # headline result, for its error
    ms_per_step = wall * 1e3 / args.steps
    taps = counts["taps"]
    value = taps / (ms_per_step / 1e3)
    rirs_batched = n_rirs / (ms_per_step / 1e3)
    k_ms = float(np.mean(launch_ms))

    res = {"metric": METRIC, "value": value, "unit": "taps/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": DTYPES[args.precision], "data": "synthetic",
           "config": {"workload": "c1: 1024 seeded shoebox rooms x 8 mics, 16 kHz, RIR 0.8*RT60*fs, "
                                  "81-tap Hann-windowed sinc, time-bounded image sets",
                      "rooms": args.rooms, "rirs": n_rirs, "taps_per_step": taps,
                      "records_per_step": counts["records"], "images_tested_per_step": counts["images"],
                      "precision": ["fp32", "fp16_lut", "fp32_split", "fp32_atomic", "fp32_direct"][args.precision],
                      "tuning": dict(H.get_tuning(), tuning_s=tune_s)},
           "rirs_per_s_batched": rirs_batched}

    # roofline of the segment kernel (the launch is one graph: upload + prologue + segments)
    achieved = FLOPS_PER_TAP * taps / (k_ms / 1e3) / 1e12
    kernel = "ism_moments" if args.precision in (0, 2) else "ism_segments"
    traffic = measured_traffic(kernel)
    res["roofline"] = {"bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFLOPS,
                       "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK_TFLOPS, "traffic": traffic,
                       "basis": "algorithmic: 12 flops per tap of the direct per-tap method (the work the "
                                "output represents), not the instructions this kernel issues, so frac can pass 1: "
                                "the moment kernel spends about 1/13 of those flops per tap (9 moments per "
                                "record, one shared filter per output sample); see 'executed'",
                       "kernel": kernel, "launch_ms": k_ms, "launch_ms_min": float(np.min(launch_ms)),
                       "launch_ms_median": float(np.median(launch_ms)),
                       "flops_per_tap": FLOPS_PER_TAP, "taps_per_launch": taps}
    # what the kernel executes (committed counters of the same source), beside the nominal rate
    cc = committed_counters(kernel)
    if cc and "executed" in cc:
        ex = cc["executed"]
        e = {"fp64_tflops": ex["fp64_flops_per_launch"] / (k_ms / 1e3) / 1e12, "fp64_peak_tflops": 78.6,
             "fp64_frac": ex["fp64_flops_per_launch"] / (k_ms / 1e3) / 1e12 / 78.6,
             "valu_issue_fraction": ex["valu_issue_fraction"],
             "note": "FP64 flops counted by rocprofv3 per launch / this run's launch time; VALU issue "
                     "fraction = VALU wave-instructions x 4 cycles / (1024 SIMDs x kernel cycles)"}
        for k in ("fp32_flops_per_launch", "lds_busy_fraction", "lds_bank_conflict_share", "wait_fraction",
                  "profile_kernel_ms", "source_hash"):
            if k in ex:
                e[k] = ex[k]
        if "fp32_flops_per_launch" in ex:
            e["fp32_tflops"] = ex["fp32_flops_per_launch"] / (k_ms / 1e3) / 1e12
        res["roofline"]["executed"] = e

    # plain: the same kernels launched once per room, host loop, one stream, launched directly
    # (no graph capture: a graph is keyed to the upload size, which changes from room to room)
    if not args.no_plain:
        saved_tuning = H.get_tuning()
        H.set_tuning(graphs=0)
        H.set_autotune(False)   # the batch's tuned segment length, no tuning inside the timed loop
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
        H.set_tuning(graphs=saved_tuning["graphs"])
        H.set_autotune(bool(saved_tuning["autotune"]))
        res["rirs_per_s_plain"] = n_rirs / plain_s
        res["taps_per_s_plain"] = taps / plain_s
        res["batched_vs_plain"] = rirs_batched / res["rirs_per_s_plain"]

    # ablation: the same batch with every tap evaluated (per-tap kernel)
    if not args.no_ablation and args.precision == 0:
        ms = _time_it(torch, lambda: H.rir_batch(batch, precision=ism.PREC_FP32_DIRECT, out=out, rooms=rooms), reps=3)
        res["ablation_fp32_direct"] = {"ms": ms, "taps_per_s": H.last_counts()["taps"] / (ms / 1e3),
                                       "kernel": "ism_segments"}
        # the paper's own 7th-order Lagrange filter (8 taps) on the same batch
        lb = dict(batch)
        lb["fd_taps"] = 8
        ms = _time_it(torch, lambda: H.rir_batch(lb, precision=ism.PREC_FP32, out=out, rooms=rooms), reps=3)
        res["lagrange_fd8"] = {"ms": ms, "taps_per_s": H.last_counts()["taps"] / (ms / 1e3),
                               "rirs_per_s": n_rirs / (ms / 1e3), "kernel": "ism_moments"}

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
        if not args.no_cpu_baseline:   # the same RIR by the FP64 oracle on one host core, and its error
            import oracle
            t = time.perf_counter()
            ref, st = oracle.rir(c0["L"][0], c0["beta"][0], c0["src"][0], c0["mics"][0], c0["fs"], c0["c"], 10, 0,
                                 4096, 81)
            dt = time.perf_counter() - t
            o1h = o1.cpu().numpy()[0].astype(np.float64)
            res["latency_ms_single_rir"]["cpu_oracle_ms_one_core"] = dt * 1e3
            res["latency_ms_single_rir"]["max_err_over_peak"] = float(np.abs(o1h - ref).max() / np.abs(ref).max())
    extras = set() if args.no_extras else {e.strip() for e in args.extras.split(",") if e.strip()}
    if extras:
        res["extras"] = {}
        if "c3" in extras:
            res["extras"]["c3_precision"] = bench_c3(H, torch, with_errors=not args.no_cpu_baseline)
        if "c0x" in extras:
            res["extras"]["c0_replicated"] = bench_c0_replicated(H, torch, with_errors=not args.no_cpu_baseline)
        if "c4" in extras:
            res["extras"]["c4_convolution"] = bench_c4(H, torch, with_errors=not args.no_cpu_baseline,
                                                       two_streams=not args.no_two_streams)
        if "paper" in extras:
            res["extras"]["paper_room1_dataset"] = bench_paper(H, torch)
        if "c2" in extras:
            res["extras"]["c2_serving"] = bench_c2(torch, args.serve_requests, batched_taps_per_s=value,
                                                  with_oracle=not args.no_cpu_baseline)
        if "beamlearning" in extras:
            bl = bench_beamlearning(H, torch)
            if not args.no_cpu_baseline:
                bl["cpu_baseline"] = cpu_baseline_beamlearning()
            res["extras"]["beamlearning_forward"] = bl
        if "rtfit" in extras:
            res["extras"]["rt_fit"] = bench_rt_fit(H, torch)
    H.close()

    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(batch, gpu=gpu_out, total_taps=taps)
        if "gpu_vs_oracle" in res["cpu_baseline"]:
            res["config"]["max_err_over_peak"] = res["cpu_baseline"]["gpu_vs_oracle"]["max_err_over_peak"]
    print(json.dumps(res))


if __name__ == "__main__":
    main()
