"""Serving engine scheduler on the CPU (mock executor: no device work).
Checks admission by HBM budget, strict FIFO order, backpressure through
release, stats, and argument errors."""
import time

import numpy as np
import pytest

from paper_2104_13347_amd import ism, scenes


def _room(M=4, L=(5.0, 4.0, 3.0), n=1600):
    mics = np.array([[2.0 + 0.05 * k, 1.5, 1.2] for k in range(M)])
    return dict(L=L, beta=[0.8] * 6, src=[1.0, 2.0, 1.5], mics=mics, rir_len=n)


def _submit(S, r):
    return S.submit(r["L"], r["beta"], r["src"], r["mics"], r["rir_len"], 16000.0, 343.0, 81)


def _wait(S, t, timeout=10.0):
    t0 = time.time()
    while time.time() - t0 < timeout:
        st, _, lat = S.poll(t)
        if st in ("done", "failed"):
            return st, lat
        time.sleep(0.001)
    raise AssertionError("timeout")


def test_budget_admission_and_backpressure():
    # pool holds exactly two 4 x 1600 outputs (25.6 kB each)
    S = ism.Server(n_lanes=2, hbm_budget_bytes=2 * 25600, max_batch_rooms=8, mock=True)
    try:
        ts = [_submit(S, _room()) for _ in range(5)]
        for t in ts[:2]:
            assert _wait(S, t)[0] == "done"
        time.sleep(0.05)
        # nothing released: the third cannot be admitted
        assert S.poll(ts[2])[0] == "queued"
        st = S.stats()
        assert st["pool_peak_bytes"] <= st["pool_bytes"]
        S.release(ts[0])
        assert _wait(S, ts[2])[0] == "done"
        assert S.poll(ts[3])[0] == "queued"
        for t in ts[1:3]:
            S.release(t)
        for t in ts[3:]:
            assert _wait(S, t)[0] == "done"
            S.release(t)
        st = S.stats()
        assert st["submitted"] == 5 and st["done"] == 5 and st["queued"] == 0
    finally:
        S.close()


def test_fifo_no_overtaking():
    # a large request at the head is not overtaken by later small ones that would fit
    S = ism.Server(n_lanes=1, hbm_budget_bytes=4 * 4 * 6000, max_batch_rooms=1, mock=True)
    try:
        small = _room(M=4, n=1000)
        big = _room(M=4, n=6000)
        a = _submit(S, small)
        assert _wait(S, a)[0] == "done"      # holds 16 kB of 96 kB
        b = _submit(S, big)                  # needs all 96 kB: waits for a's release
        c = _submit(S, small)
        time.sleep(0.05)
        assert S.poll(b)[0] == "queued" and S.poll(c)[0] == "queued"
        S.release(a)
        assert _wait(S, b)[0] == "done"
        assert S.poll(c)[0] == "queued"
        S.release(b)
        assert _wait(S, c)[0] == "done"
        S.release(c)
    finally:
        S.close()


def test_replay_mock_latencies():
    S = ism.Server(n_lanes=4, hbm_budget_bytes=1 << 30, max_batch_rooms=16, mock=True)
    try:
        reqs, gaps, meta = scenes.c2(n_requests=200)
        b = scenes.pack(reqs, meta["fs"], meta["c"], meta["fd_taps"], meta["order_mode"], "c2")
        lat, wall = S.replay(b, np.cumsum(gaps) * 1e-3)
        assert np.all(lat > 0) and wall > 0
        st = S.stats()
        assert st["done"] == 200 and st["batches"] >= 1
    finally:
        S.close()


def test_server_errors():
    S = ism.Server(n_lanes=1, hbm_budget_bytes=1 << 20, max_batch_rooms=4, mock=True)
    try:
        with pytest.raises(ism.IsmError):            # larger than the whole budget
            _submit(S, _room(M=32, n=16000))
        r = _room()
        r["src"] = [0.0, 2.0, 1.5]
        with pytest.raises(ism.IsmError):            # source on a wall
            _submit(S, r)
        with pytest.raises(ism.IsmError):
            S.release(12345)
        t = _submit(S, _room())
        _wait(S, t)
        with pytest.raises(ism.IsmError):            # no device memory in mock mode
            S.result(t, 4, 1600) if False else S._check(S.lib.ism_server_copy_result(S.s, t, None, None))
        S.release(t)
    finally:
        S.close()
    with pytest.raises(ism.IsmError):
        ism.Server(n_lanes=0, mock=True)
