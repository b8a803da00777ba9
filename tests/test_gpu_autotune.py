"""GPU checks of the launch autotuner (batched form of section II.A's RIR computation):
the first batch of a shape bucket is tuned and its result meets the bar against the
FP64 oracle; later batches of the bucket reuse the cached choice; the moment kernel is
never offered a segment longer than it takes; and the tuned configuration is not slower
than the default one on the 1024-room distribution and the 48 kHz workload (subsets)."""
import sys

import numpy as np
import pytest

import oracle
from paper_2104_13347_amd import ism, scenes

pytestmark = pytest.mark.gpu
TOL_FP32 = 1e-5


def _say(msg):
    sys.stdout.write(msg + "\n")
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _errors(batch, gpu, rirs):
    ref, _ = oracle.rir_list(batch, rirs)
    e = []
    for r, m in rirs:
        L = int(batch["rir_len"][r])
        o = int(batch["out_offset"][r]) + m * L
        e.append(np.abs(gpu[o:o + L] - ref[o:o + L]).max() / np.abs(ref[o:o + L]).max())
    return np.array(e)


def test_autotune_on_first_use_of_a_bucket(torch_cuda):
    torch = torch_cuda
    h = ism.Handle()
    try:
        h.set_autotune(True)
        b = scenes.c1(n_rooms=16)
        out = h.rir_batch(b)          # tuned here; out holds the winner's result
        torch.cuda.synchronize()
        t = h.get_tuning()
        _say(f"tuned {t}")
        assert t["tuned_buckets"] >= 1 and t["seg_len"] in (256, 512, 1024) and t["tuned_ms"] > 0
        rirs = [(r, (3 * r) % 8) for r in range(16)]
        assert _errors(b, out.cpu().numpy(), rirs).max() <= TOL_FP32
        n_before = t["tuned_buckets"]
        again = h.rir_batch(b)        # same bucket: cached, bitwise the same launch
        torch.cuda.synchronize()
        assert h.get_tuning()["tuned_buckets"] == n_before
        assert torch.equal(out, again)
        c = scenes.subset(scenes.c3(), [0])   # another bucket (48 kHz, 16 mics)
        h.rir_batch(c)
        torch.cuda.synchronize()
        assert h.get_tuning()["tuned_buckets"] == n_before + 1
    finally:
        h.close()


def test_batch_size_is_part_of_the_bucket(torch_cuda):
    # one RIR and 4096 RIRs of the same room shape are tuned separately, and the large
    # batch's tuned configuration is not slower than the small one's choice on it
    torch = torch_cuda
    h = ism.Handle()
    try:
        h.set_autotune(True)
        big = scenes.c0_replicated()
        one = scenes.subset(big, [0])
        h.rir_batch(one)
        torch.cuda.synchronize()
        t1 = h.get_tuning()
        out = torch.empty(int(big["out_size"]), dtype=torch.float32, device="cuda")
        h.rir_batch(big, out=out)
        torch.cuda.synchronize()
        t2 = h.get_tuning()
        _say(f"one RIR {t1}, 4096 RIRs {t2}")
        assert t2["tuned_buckets"] == t1["tuned_buckets"] + 1
        tuned = _time(torch, h, big, out)
        h.set_autotune(False)
        h.set_tuning(seg_len=t1["seg_len"])
        small_choice = _time(torch, h, big, out)
        _say(f"4096 RIRs: tuned {tuned:.3f} ms, with the one-RIR choice {small_choice:.3f} ms")
        assert tuned <= small_choice * 1.05
    finally:
        h.close()


def _time(torch, h, b, out, reps=3):
    ts = []
    for _ in range(reps + 1):
        a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        h.rir_batch(b, out=out)
        z.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(z))
    return float(np.median(ts[1:]))


@pytest.mark.parametrize("workload", ["c1_256_rooms", "c3_8_rooms"])
def test_tuned_is_not_slower_than_default(torch_cuda, workload):
    torch = torch_cuda
    b = scenes.subset(scenes.c1(), list(range(256))) if workload == "c1_256_rooms" else \
        scenes.subset(scenes.c3(), list(range(8)))
    out = torch.empty(int(b["out_size"]), dtype=torch.float32, device="cuda")
    d = ism.Handle()
    h = ism.Handle()
    try:
        t_def = _time(torch, d, b, out)
        best = h.autotune(b, out=out)
        t_tuned = _time(torch, h, b, out)
        _say(f"{workload}: default (seg 1024) {t_def:.3f} ms, tuned (seg {best}) {t_tuned:.3f} ms")
        assert best <= 1024               # the moment kernel's limit
        assert t_tuned <= 1.05 * t_def    # timing noise margin
    finally:
        d.close()
        h.close()
