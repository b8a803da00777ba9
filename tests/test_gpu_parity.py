"""GPU parity: the HIP path through the C-ABI against the FP64 oracle.

Bar (per RIR): max |gpu - oracle| <= 1e-5 * max |oracle| for the FP32 paths (the
moment evaluation and the per-tap direct one),
<= 2e-3 * max |oracle| for the FP16 table variant; tap counts (integers) equal
exactly; repeated and batched runs bitwise equal.
"""
import math
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2104_13347_amd import ism, scenes

pytestmark = pytest.mark.gpu

TOL_FP32 = 1e-5
TOL_LUT = 2e-3


def _say(msg):
    sys.stdout.write(msg + "\n")
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def H(torch_cuda):
    h = ism.Handle()
    yield h
    h.close()


def oracle_batch(batch, rirs=None, nthreads=None):
    if rirs is None:
        rirs = [(r, m) for r in range(len(batch["rir_len"])) for m in range(int(batch["n_mics"][r]))]
    out, taps = oracle.rir_list(batch, rirs, nthreads=nthreads)
    return out, taps, rirs


def rel_errors(batch, gpu, ref, rirs):
    errs = []
    for r, m in rirs:
        L = int(batch["rir_len"][r])
        o = int(batch["out_offset"][r]) + m * L
        a, b = gpu[o:o + L].astype(np.float64), ref[o:o + L]
        peak = float(np.max(np.abs(b)))
        errs.append(float(np.max(np.abs(a - b))) / peak if peak > 0 else float(np.max(np.abs(a))))
    return np.array(errs)


def run(H, batch, precision=ism.PREC_FP32, seg_len=None):
    import torch
    if seg_len:
        H.set_tuning(seg_len=seg_len)
    out = H.rir_batch(batch, precision=precision)
    torch.cuda.synchronize()
    res = out.cpu().numpy()
    cnt = H.last_counts()
    H.set_tuning(seg_len=1024)
    return res, cnt


# ------------------------------------------------------------------ configurations
@pytest.mark.parametrize("precision", [ism.PREC_FP32, ism.PREC_FP32_DIRECT])
@pytest.mark.parametrize("mode", [ism.ORDER_INDEX_L1, ism.ORDER_REFLECTIONS])
@pytest.mark.parametrize("seg_len", [64, 1024, 2048])
def test_c0_single_room(H, mode, seg_len, precision):
    b = scenes.c0()
    b["order_mode"] = mode
    _say(f"c0 mode={mode} seg_len={seg_len} precision={precision}")
    gpu, cnt = run(H, b, precision=precision, seg_len=seg_len)
    ref, taps, rirs = oracle_batch(b)
    err = rel_errors(b, gpu, ref, rirs)
    assert err.max() <= TOL_FP32, err
    assert cnt["taps"] == taps == (1005974 if mode == 0 else 126441)


@pytest.mark.parametrize("taps,rir_len,seg_len", [(9, 64, 64), (9, 300, 64), (21, 333, 128), (1, 200, 64),
                                                 (81, 700, 192), (127, 900, 256), (255, 1000, 512)])
def test_tiny_rooms_all_kernel_variants(H, taps, rir_len, seg_len):
    b = scenes.tiny(seed=taps + rir_len, n_rooms=3, rir_len=rir_len, M=3, taps=taps)
    _say(f"tiny taps={taps} len={rir_len} seg={seg_len}")
    gpu, cnt = run(H, b, seg_len=seg_len)
    ref, ntaps, rirs = oracle_batch(b)
    err = rel_errors(b, gpu, ref, rirs)
    assert err.max() <= TOL_FP32, err
    assert cnt["taps"] == ntaps


@pytest.mark.parametrize("precision", [ism.PREC_FP32, ism.PREC_FP32_DIRECT])
def test_c1_sixteen_rooms(H, precision):
    full = scenes.c1()
    b = scenes.subset(full, range(16))
    _say(f"c1 16 rooms precision={precision}")
    gpu, cnt = run(H, b, precision=precision)
    ref, taps, rirs = oracle_batch(b)
    err = rel_errors(b, gpu, ref, rirs)
    _say(f"c1 16 rooms max err {err.max():.3e}")
    assert err.max() <= TOL_FP32
    assert cnt["taps"] == taps


def test_c1_full_batch_sampled(H):
    # the 1024-room batch in the benchmark's launch configuration; 24 RIRs checked one by one
    b = scenes.c1()
    _say("c1 full batch")
    gpu, cnt = run(H, b)
    rng = np.random.default_rng(5)
    rooms = rng.choice(len(b["rir_len"]), size=24, replace=False)
    rirs = [(int(r), int(rng.integers(0, 8))) for r in rooms]
    ref, _, _ = oracle_batch(b, rirs)
    err = rel_errors(b, gpu, ref, rirs)
    _say(f"c1 sampled max err {err.max():.3e}")
    assert err.max() <= TOL_FP32
    assert np.all(np.isfinite(gpu))
    # every RIR has its direct path: nonzero energy in every output row
    assert cnt["taps"] > 0.9e11


def test_c0_replicated_full_batch_sampled(H):
    # the single-RIR room as 4096 rooms (the benchmark's launch): 16 RIRs against the oracle
    # one by one, and the exact tap count of those 16 rooms run as a batch of their own
    b = scenes.c0_replicated()
    _say("c0 replicated full batch")
    gpu, cnt = run(H, b)
    rirs = [(r, 0) for r in range(0, 4096, 256)]
    ref, taps, _ = oracle_batch(b, rirs)
    err = rel_errors(b, gpu, ref, rirs)
    _say(f"c0 replicated sampled max err {err.max():.3e}")
    assert err.max() <= TOL_FP32
    assert np.all(np.isfinite(gpu))
    _, cnt16 = run(H, scenes.subset(b, [r for r, _ in rirs]))
    assert cnt16["taps"] == taps


def _order_mix(mode, fd_taps, seed=31):
    # 12 rooms of 2.5-4 m, random per-wall beta, 3 microphones, 1024 or 2048 samples at
    # 16 kHz, image sets bounded by orders 0, 1, 2, 5 and 10 or by time (-1) in one batch
    rng = np.random.default_rng(seed)
    rooms = []
    for i, order in enumerate([0, 1, 2, 5, 10, -1] * 2):
        L = np.array([rng.uniform(2.5, 4.0), rng.uniform(2.5, 4.0), rng.uniform(2.5, 3.0)])
        src = rng.uniform(0.3, 1.0, 3) * (L - 0.6) + 0.3
        mics = np.array([rng.uniform(0.0, 1.0, 3) * (L - 0.6) + 0.3 for _ in range(3)])
        rooms.append({"L": L, "beta": rng.uniform(0.4, 0.95, 6), "src": src, "mics": mics, "max_order": order,
                      "rir_len": 1024 if i % 2 else 2048})
    return scenes.pack(rooms, 16000.0, scenes.C_SOUND, fd_taps, mode, "order-mix")


@pytest.mark.parametrize("precision", [ism.PREC_FP32, ism.PREC_FP32_DIRECT])
@pytest.mark.parametrize("fd_taps", [81, 8])
@pytest.mark.parametrize("mode", [ism.ORDER_INDEX_L1, ism.ORDER_REFLECTIONS])
def test_order_bounded_batch(H, mode, fd_taps, precision):
    # order bounds in both counting modes (index L1 and reflections), mixed with
    # time-bounded rooms in one launch; every RIR against the oracle, exact tap count
    b = _order_mix(mode, fd_taps)
    _say(f"order mix mode={mode} fd_taps={fd_taps} precision={precision}")
    if fd_taps == 8 and precision == ism.PREC_FP32_DIRECT:
        # the Lagrange filter runs in the moment form (its per-tap form serves only rooms
        # past the moment kernel's tables); the per-tap precision mode is refused for it
        with pytest.raises(ism.IsmError):
            run(H, b, precision=precision)
        return
    gpu, cnt = run(H, b, precision=precision)
    ref, taps, rirs = oracle_batch(b)
    err = rel_errors(b, gpu, ref, rirs)
    _say(f"order mix max err {err.max():.3e}, taps {cnt['taps']} / {taps}")
    assert err.max() <= TOL_FP32
    assert cnt["taps"] == taps


@pytest.mark.parametrize("fd_taps", [81, 8])
def test_walls_of_zero_and_unit_reflection(H, fd_taps):
    # walls that absorb everything (beta = 0: beta^0 = 1 for the images that never hit
    # them) beside fully reflecting walls (beta = 1) and ordinary ones, time-bounded, in
    # one launch; every RIR against the oracle, exact tap count
    patterns = [[0.0, 1.0, 0.5, 0.0, 1.0, 0.7], [1.0] * 4 + [0.0, 0.0], [0.0, 0.0, 1.0, 1.0, 0.9, 0.9],
                [1.0] * 6, [0.0] * 5 + [1.0], [0.3, 1.0, 0.0, 0.8, 1.0, 0.0]]
    rng = np.random.default_rng(41)
    rooms = []
    for i, beta in enumerate(patterns):
        L = np.array([rng.uniform(3.0, 5.0), rng.uniform(3.0, 4.0), rng.uniform(2.5, 3.0)])
        src = rng.uniform(0.2, 0.8, 3) * L
        mics = np.array([rng.uniform(0.2, 0.8, 3) * L for _ in range(2)])
        rooms.append({"L": L, "beta": beta, "src": src, "mics": mics, "max_order": -1, "rir_len": 600 + 200 * i})
    b = scenes.pack(rooms, 16000.0, scenes.C_SOUND, fd_taps, ism.ORDER_INDEX_L1, "walls")
    gpu, cnt = run(H, b)
    ref, taps, rirs = oracle_batch(b)
    err = rel_errors(b, gpu, ref, rirs)
    _say(f"zero/unit walls fd_taps={fd_taps}: max err {err.max():.3e}, taps {cnt['taps']} / {taps}")
    assert err.max() <= TOL_FP32
    assert cnt["taps"] == taps


@pytest.mark.parametrize("fd_taps", [81, 8])
def test_microphone_next_to_the_source(H, fd_taps):
    # source-microphone distances of 1 mm, 1 cm and 10 cm: the direct path's gain (up to
    # 80) sets the item's fixed-point scale far above every reflection; every RIR against
    # the oracle, exact tap count
    src = np.array([1.7, 2.2, 1.4])
    rooms = [{"L": (4.0, 5.0, 3.0), "beta": (0.8,) * 6, "src": src, "max_order": -1, "rir_len": 1500,
              "mics": [src + np.array([d, 0.0, 0.0]), src + np.array([0.0, -d, d])]} for d in (1e-3, 1e-2, 1e-1)]
    b = scenes.pack(rooms, 16000.0, scenes.C_SOUND, fd_taps, ism.ORDER_INDEX_L1, "near")
    gpu, cnt = run(H, b)
    ref, taps, rirs = oracle_batch(b)
    err = rel_errors(b, gpu, ref, rirs)
    _say(f"near field fd_taps={fd_taps}: max err {err.max():.3e}, taps {cnt['taps']} / {taps}")
    assert err.max() <= TOL_FP32
    assert cnt["taps"] == taps


def test_c3_precision_variants(H):
    b = scenes.subset(scenes.c3(), [0, 1])
    ref, taps, rirs = oracle_batch(b)
    res = {}
    for prec, name in [(ism.PREC_FP32, "fp32"), (ism.PREC_FP32_DIRECT, "direct"), (ism.PREC_FP32_ATOMIC, "atomic"),
                       (ism.PREC_FP16_LUT, "lut"), (ism.PREC_FP32_SPLIT, "split32")]:
        _say(f"c3 {name}")
        gpu, cnt = run(H, b, precision=prec)
        res[name] = rel_errors(b, gpu, ref, rirs).max()
        if name != "split32":
            assert cnt["taps"] == taps
    _say(f"c3 errors {res}")
    assert res["fp32"] <= TOL_FP32
    assert res["direct"] <= TOL_FP32
    assert res["atomic"] <= TOL_FP32
    assert res["lut"] <= TOL_LUT
    assert res["split32"] >= res["fp32"]


def test_autotune_picks_a_candidate_and_keeps_results(H):
    # the autotuner times each segment length on the batch and keeps the fastest; the batch
    # then runs with it, and its RIRs still meet the bar against the oracle
    import torch
    b = scenes.c1(n_rooms=12)
    best = H.autotune(b, candidates=[256, 512, 1024])
    torch.cuda.synchronize()
    _say(f"autotune best seg_len {best}")
    assert best in (256, 512, 1024)
    assert H.get_tuning()["seg_len"] == best
    out = H.rir_batch(b)
    torch.cuda.synchronize()
    gpu = out.cpu().numpy()
    rirs = [(r, r % 8) for r in range(12)]
    ref, _, _ = oracle_batch(b, rirs)
    assert rel_errors(b, gpu, ref, rirs).max() <= TOL_FP32
    H.set_tuning(seg_len=1024)


def test_c3_all_rooms_sampled(H):
    # the 48 kHz workload in its benchmark launch (64 rooms x 16 mics, 72 000 samples,
    # 127 taps); one microphone of every room (a different one per room) against the oracle
    b = scenes.c3()
    gpu, _ = run(H, b)
    rirs = [(r, r % 16) for r in range(64)]
    _say("c3 all rooms: oracle")
    ref, _, _ = oracle_batch(b, rirs, nthreads=min(16, os.cpu_count() or 1))
    err = rel_errors(b, gpu, ref, rirs)
    _say(f"c3 all rooms: max err {err.max():.3e} (room {int(err.argmax())})")
    assert err.max() <= TOL_FP32
    assert np.all(np.isfinite(gpu))


def test_absorbing_rooms_late_segments(H):
    # Strongly absorbing walls (beta 0.02 .. 0.3, and one room with beta = 0) and long RIRs:
    # in late segments nearly all records have gains far below the item's scale, so the
    # filter's bin scale comes from the record count rather than the largest bin.
    rng = np.random.default_rng(31)
    rooms = []
    for i in range(4):
        L = np.array([rng.uniform(3, 6), rng.uniform(3, 5), rng.uniform(2.5, 3.5)])
        beta = rng.uniform(0.02, 0.3, size=6) if i < 3 else np.zeros(6)
        src = L * rng.uniform(0.2, 0.8, size=3)
        mics = L * rng.uniform(0.2, 0.8, size=(2, 3))
        rooms.append({"L": L, "beta": beta, "src": src, "mics": mics, "max_order": -1, "rir_len": 3000})
    b = scenes.pack(rooms, 16000.0, scenes.C_SOUND, 81, ism.ORDER_INDEX_L1, "absorbing")
    _say("absorbing rooms")
    gpu, cnt = run(H, b)
    ref, taps, rirs = oracle_batch(b)
    assert np.all(np.isfinite(gpu))
    err = rel_errors(b, gpu, ref, rirs)
    _say(f"absorbing max err {err.max():.3e}")
    assert err.max() <= TOL_FP32
    assert cnt["taps"] == taps


# ------------------------------------------------------------------ determinism
def test_repeat_and_batched_vs_per_room_bitwise(H):
    import torch
    b = scenes.subset(scenes.c1(), range(6))
    a1, _ = run(H, b)
    a2, _ = run(H, b)
    assert np.array_equal(a1, a2)
    for r in range(6):
        o, M, L = int(b["out_offset"][r]), int(b["n_mics"][r]), int(b["rir_len"][r])
        mo = int(b["mic_offset"][r])
        single = H.rir(b["L"][r], b["beta"][r], b["src"][r], b["mics"][mo:mo + M], b["fs"], b["c"], -1, L, 81)
        torch.cuda.synchronize()
        assert np.array_equal(single.cpu().numpy().ravel(), a1[o:o + M * L])


def test_graph_replay_equals_direct_launch(H):
    import torch
    b = scenes.subset(scenes.c1(), range(4))
    H.set_tuning(graphs=0)
    a, _ = run(H, b)
    H.set_tuning(graphs=1)
    outs = []
    for _ in range(3):           # replays with eager work in between
        outs.append(run(H, b)[0])
        torch.zeros(1 << 20, device="cuda").sum().item()
    for o in outs:
        assert np.array_equal(o, a)


# ------------------------------------------------------------------ edge cases
def test_edge_cases(H, torch_cuda):
    torch = torch_cuda
    # beta = 0: direct path only; integer delay: Kronecker impulse
    out = H.rir([2.0, 2.0, 4.0], [0.0] * 6, [1.0, 1.0, 1.0], [[1.0, 1.0, 3.5]], 136.0, 340.0, -1, 32, 9)
    torch.cuda.synchronize()
    o = out.cpu().numpy()[0]
    g = 1.0 / (4.0 * math.pi * 2.5)
    assert abs(o[1] - g) <= 1e-5 * g
    assert np.max(np.abs(np.delete(o, 1))) <= 1e-5 * g
    # rir_len = 1, max_order = 0 (direct only), microphones on walls
    for L, mics, N, n in [([5.0, 4.0, 3.0], [[5.0, 0.0, 3.0], [2.0, 2.0, 0.0]], 0, 1),
                          ([5.0, 4.0, 3.0], [[5.0, 0.0, 3.0]], 3, 777)]:
        out = H.rir(L, [0.6] * 6, [1.3, 2.1, 1.5], mics, 16000.0, 343.0, N, n, 81)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        for m, mic in enumerate(mics):
            ref, _ = oracle.rir(L, [0.6] * 6, [1.3, 2.1, 1.5], mic, 16000.0, 343.0, N, 0, n, 81)
            peak = max(np.max(np.abs(ref)), 1e-30)
            assert np.max(np.abs(got[m] - ref)) <= 1e-5 * peak
    # empty batch is a no-op
    e = scenes.pack([], 16000.0, 343.0, 81, 0, "empty")
    assert H.lib.ism_rir_batch(H.h, 0, None, None, 16000.0, 343.0, 81, 0, 0, None, None) == 0


# ------------------------------------------------------------------ the paper's Lagrange filter
@pytest.mark.parametrize("mode", [ism.ORDER_INDEX_L1, ism.ORDER_REFLECTIONS])
@pytest.mark.parametrize("seg_len", [64, 1024, 2048])
def test_c0_lagrange(H, mode, seg_len):
    b = scenes.c0()
    b["order_mode"] = mode
    b["fd_taps"] = 8
    _say(f"c0 lagrange mode={mode} seg_len={seg_len}")
    gpu, cnt = run(H, b, seg_len=seg_len)
    ref, taps, rirs = oracle_batch(b)
    err = rel_errors(b, gpu, ref, rirs)
    _say(f"c0 lagrange max err {err.max():.3e}")
    assert err.max() <= TOL_FP32, err
    assert cnt["taps"] == taps


def test_c1_lagrange_sixteen_rooms_and_tiny_rooms(H):
    b = scenes.subset(scenes.c1(), range(16))
    b["fd_taps"] = 8
    _say("c1 16 rooms lagrange")
    gpu, cnt = run(H, b)
    ref, taps, rirs = oracle_batch(b)
    err = rel_errors(b, gpu, ref, rirs)
    _say(f"c1 lagrange max err {err.max():.3e}")
    assert err.max() <= TOL_FP32
    assert cnt["taps"] == taps
    t = scenes.tiny(seed=77, n_rooms=3, rir_len=300, M=3, taps=9)
    t["fd_taps"] = 8
    gpu, cnt = run(H, t, seg_len=64)
    ref, taps, rirs = oracle_batch(t)
    assert rel_errors(t, gpu, ref, rirs).max() <= TOL_FP32
    assert cnt["taps"] == taps


def test_paper_room_dataset_sources(H):
    # the paper's room (7 x 10 x 3.7 m, RT 0.5 s, 7-microphone array, torus sources): three
    # source positions, both filters, against the oracle
    for taps in (8, 81):
        b = scenes.paper_room1(n_sources=3, fd_taps=taps)
        _say(f"paper room taps={taps}")
        gpu, cnt = run(H, b)
        ref, ntaps, rirs = oracle_batch(b)
        err = rel_errors(b, gpu, ref, rirs)
        _say(f"paper room taps={taps} max err {err.max():.3e}")
        assert err.max() <= TOL_FP32
        assert cnt["taps"] == ntaps


@pytest.mark.parametrize("fd_taps", [81, 8])
def test_long_rir_in_a_thin_room_uses_the_per_tap_kernel(H, torch_cuda, fd_taps):
    # wall exponents up to about 130 (a 0.3 m room height, 3500 samples): the moment kernel
    # holds at most 128 in LDS, so both the windowed sinc and the paper's Lagrange filter
    # fall back to the per-tap kernel
    torch = torch_cuda
    L, beta, s, m = [3.0, 3.0, 0.3], [0.6] * 6, [1.0, 1.2, 0.1], [[2.1, 1.7, 0.2], [0.4, 2.6, 0.15]]
    out = H.rir(L, beta, s, m, 16000.0, 343.0, -1, 3500, fd_taps)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    taps = 0
    for k in range(2):
        ref, st = oracle.rir(L, beta, s, m[k], 16000.0, 343.0, -1, 0, 3500, fd_taps)
        taps += st["taps"]
        err = np.max(np.abs(got[k] - ref)) / np.max(np.abs(ref))
        _say(f"thin room fd_taps {fd_taps} mic {k}: err {err:.2e}")
        assert err <= TOL_FP32
    assert H.last_counts()["taps"] == taps


def test_lagrange_per_tap_kernel_tiny_rooms_and_kronecker(H, torch_cuda):
    # the per-tap Lagrange path on thin tiny rooms (every tap of the image sum against the
    # oracle) and an integer delay (the Kronecker impulse: one tap of weight g)
    torch = torch_cuda
    rng = np.random.default_rng(44)
    for i in range(3):
        L = [rng.uniform(1.0, 2.0), rng.uniform(1.0, 2.0), rng.uniform(0.12, 0.2)]
        beta = list(rng.uniform(0.3, 0.9, 6))
        s = [L[0] * 0.3, L[1] * 0.6, L[2] * 0.4]
        m = [[L[0] * 0.7, L[1] * 0.2, L[2] * 0.7]]
        n = 2600
        out = H.rir(L, beta, s, m, 16000.0, 343.0, -1, n, 8)
        torch.cuda.synchronize()
        ref, st = oracle.rir(L, beta, s, m[0], 16000.0, 343.0, -1, 0, n, 8)
        err = np.max(np.abs(out.cpu().numpy()[0] - ref)) / np.max(np.abs(ref))
        _say(f"thin tiny room {i}: err {err:.2e}, taps {st['taps']}")
        assert err <= TOL_FP32 and H.last_counts()["taps"] == st["taps"]
    # Kronecker: beta 0, integer delay tau = 1 (s = (1,1,1), r = (1,1,3.5), c = 340, fs = 136),
    # in a room thin enough in x for the per-tap kernel (the direct path is the only image)
    out = H.rir([0.05, 2.0, 4.0], [0.0] * 6, [0.025, 1.0, 1.0], [[0.025, 1.0, 3.5]], 136.0, 340.0, -1, 4, 8)
    torch.cuda.synchronize()
    got = out.cpu().numpy()[0]
    g = 1.0 / (4.0 * math.pi * 2.5)
    assert abs(got[1] - g) <= 1e-6 * g and np.max(np.abs(np.delete(got, 1))) <= 1e-6 * g
