"""Thin ctypes binding of libism.so (C-ABI declared in include/ism.h).

Argument marshalling only: every step of the RIR path runs in the library's HIP
kernels.  torch supplies device memory (``Tensor.data_ptr()``) and streams
(``torch.cuda.current_stream().cuda_stream``).  If the library is not built the
import fails loudly; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("ISM_LIB") or os.path.join(_HERE, "libism.so")

ISM_OK, ISM_EINVAL, ISM_EDOMAIN, ISM_ENOMEM, ISM_EDEVICE, ISM_EBUSY = 0, -1, -2, -3, -4, -5
ORDER_INDEX_L1, ORDER_REFLECTIONS = 0, 1
PREC_FP32, PREC_FP16_LUT, PREC_FP32_SPLIT, PREC_FP32_ATOMIC, PREC_FP32_DIRECT = 0, 1, 2, 3, 4

# exported symbols (kept in step with include/ism.h)
EXPORTS = [
    "ism_create", "ism_destroy", "ism_strerror", "ism_last_error", "ism_version", "ism_rir",
    "ism_rir_batch", "ism_batch_plan_stats", "ism_last_counts", "ism_set_tuning", "ism_get_tuning",
    "ism_autotune", "ism_set_autotune", "ism_get_launch_tuning", "ism_convolve_batch", "ism_convolve_batch_z", "ism_normal_deviates", "ism_conv_set_timing", "ism_conv_last_timing", "ism_server_create", "ism_server_destroy", "ism_server_submit",
    "ism_server_poll", "ism_server_copy_result", "ism_server_release", "ism_server_stats", "ism_server_counters", "ism_server_last_error", "ism_server_replay",
    "ism_rt_work_bytes", "ism_rir_t30", "ism_fit_beta", "ism_rt_mean_work_bytes", "ism_fit_beta_mean",
]

ROOM_DTYPE = np.dtype([("L", np.float64, 3), ("beta", np.float64, 6), ("src", np.float64, 3),
                       ("mic_offset", np.int32), ("n_mics", np.int32), ("max_order", np.int32),
                       ("rir_len", np.int32), ("out_offset", np.int64)], align=True)
assert ROOM_DTYPE.itemsize == 120


class IsmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


_lib = None


def load():
    """Load libism.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() or "
                          "python paper_2104_13347_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    vp, dp, i32p, i64p, fp = (ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                              ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64),
                              ctypes.POINTER(ctypes.c_float))
    ci, cd = ctypes.c_int, ctypes.c_double
    L.ism_create.argtypes = [ctypes.POINTER(vp)]
    L.ism_create.restype = ci
    L.ism_destroy.argtypes = [vp]
    L.ism_destroy.restype = None
    L.ism_strerror.argtypes = [ci]
    L.ism_strerror.restype = ctypes.c_char_p
    L.ism_last_error.argtypes = [vp]
    L.ism_last_error.restype = ctypes.c_char_p
    L.ism_version.restype = ci
    L.ism_rir.argtypes = [vp, dp, dp, dp, ci, dp, cd, cd, ci, ci, ci, ci, ci, vp, vp]
    L.ism_rir.restype = ci
    L.ism_rir_batch.argtypes = [vp, ci, vp, dp, cd, cd, ci, ci, ci, vp, vp]
    L.ism_rir_batch.restype = ci
    L.ism_batch_plan_stats.argtypes = [vp, ci, vp, dp, cd, cd, ci, i64p, dp, dp]
    L.ism_batch_plan_stats.restype = ci
    L.ism_last_counts.argtypes = [vp, i64p]
    L.ism_last_counts.restype = ci
    L.ism_set_tuning.argtypes = [vp, ci, ci, ci]
    L.ism_set_tuning.restype = ci
    L.ism_get_tuning.argtypes = [vp, ctypes.POINTER(ci), ctypes.POINTER(ci), ctypes.POINTER(ci)]
    L.ism_get_tuning.restype = ci
    L.ism_autotune.argtypes = [vp, ci, vp, dp, cd, cd, ci, ci, ci, vp, vp, ctypes.POINTER(ci), ci,
                               ctypes.POINTER(ci)]
    L.ism_autotune.restype = ci
    L.ism_set_autotune.argtypes = [vp, ci]
    L.ism_set_autotune.restype = ci
    L.ism_get_launch_tuning.argtypes = [vp] + [ctypes.POINTER(ci)] * 5 + [fp]
    L.ism_get_launch_tuning.restype = ci
    L.ism_convolve_batch.argtypes = [vp, ci, ci, vp, i64p, i32p, vp, ci, ci, fp, ctypes.c_uint64, ci, vp, vp]
    L.ism_convolve_batch.restype = ci
    L.ism_convolve_batch_z.argtypes = [vp, ci, ci, vp, i64p, i32p, vp, ci, ci, fp, vp, ci, vp, vp]
    L.ism_convolve_batch_z.restype = ci
    L.ism_normal_deviates.argtypes = [vp, ci, ci, ci, ctypes.c_uint64, vp, vp]
    L.ism_normal_deviates.restype = ci
    L.ism_conv_set_timing.argtypes = [vp, ci]
    L.ism_conv_set_timing.restype = ci
    L.ism_conv_last_timing.argtypes = [vp, ctypes.POINTER(ctypes.c_float)]
    L.ism_conv_last_timing.restype = ci
    L.ism_server_create.argtypes = [ci, ctypes.c_size_t, ci, ci, ctypes.POINTER(vp)]
    L.ism_server_create.restype = ci
    L.ism_server_destroy.argtypes = [vp]
    L.ism_server_destroy.restype = None
    L.ism_server_submit.argtypes = [vp, vp, dp, cd, cd, ci, ci, ci, ctypes.POINTER(ctypes.c_uint64)]
    L.ism_server_submit.restype = ci
    L.ism_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(ci), ctypes.POINTER(vp), dp]
    L.ism_server_poll.restype = ci
    L.ism_server_copy_result.argtypes = [vp, ctypes.c_uint64, vp, vp]
    L.ism_server_copy_result.restype = ci
    L.ism_server_release.argtypes = [vp, ctypes.c_uint64]
    L.ism_server_release.restype = ci
    L.ism_server_stats.argtypes = [vp, i64p]
    L.ism_server_stats.restype = ci
    L.ism_server_counters.argtypes = [vp, i64p]
    L.ism_server_counters.restype = ci
    L.ism_server_last_error.argtypes = [vp]
    L.ism_server_last_error.restype = ctypes.c_char_p
    L.ism_server_replay.argtypes = [vp, ci, vp, dp, dp, cd, cd, ci, dp, dp]
    L.ism_server_replay.restype = ci
    L.ism_rt_work_bytes.argtypes = [ci]
    L.ism_rt_work_bytes.restype = ctypes.c_size_t
    L.ism_rir_t30.argtypes = [vp, vp, ci, cd, vp, vp]
    L.ism_rir_t30.restype = ci
    L.ism_fit_beta.argtypes = [vp, dp, dp, dp, cd, cd, ci, cd, ci, ci, vp, ctypes.c_size_t, dp, dp, vp]
    L.ism_fit_beta.restype = ci
    L.ism_rt_mean_work_bytes.argtypes = [ci, ci, ci]
    L.ism_rt_mean_work_bytes.restype = ctypes.c_size_t
    L.ism_fit_beta_mean.argtypes = [vp, dp, ci, dp, ci, dp, cd, cd, ci, cd, ci, ci, vp, ctypes.c_size_t, dp, dp, vp]
    L.ism_fit_beta_mean.restype = ci
    _lib = L
    return L


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def rooms_array(batch):
    """Pack a scene batch (see scenes.pack) into the C ism_room layout."""
    R = len(batch["rir_len"])
    r = np.zeros(R, dtype=ROOM_DTYPE)
    r["L"] = batch["L"]
    r["beta"] = batch["beta"]
    r["src"] = batch["src"]
    r["mic_offset"] = batch["mic_offset"]
    r["n_mics"] = batch["n_mics"]
    r["max_order"] = batch["max_order"]
    r["rir_len"] = batch["rir_len"]
    r["out_offset"] = batch["out_offset"]
    return r


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


def _on(stream):
    """Context in which temporaries (outputs, workspaces, contiguous copies) are allocated and
    written on the stream the library queues its work on, so the caching allocator orders
    their reuse after that work."""
    import contextlib
    import torch
    return contextlib.nullcontext() if stream is None else torch.cuda.stream(stream)


class Handle:
    """Owns an ism_handle (device buffers, pinned staging, tuning state, graphs)."""

    def __init__(self):
        self.lib = load()
        h = ctypes.c_void_p()
        rc = self.lib.ism_create(ctypes.byref(h))
        if rc != ISM_OK:
            raise IsmError(rc, "ism_create failed: " + self.lib.ism_strerror(rc).decode())
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.ism_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != ISM_OK:
            raise IsmError(rc, self.lib.ism_last_error(self.h).decode() or
                           self.lib.ism_strerror(rc).decode())

    # -- tuning
    def set_tuning(self, seg_len=0, wg_per_cu=-1, graphs=-1):
        self._check(self.lib.ism_set_tuning(self.h, int(seg_len), int(wg_per_cu), int(graphs)))

    def get_tuning(self):
        a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        self._check(self.lib.ism_get_tuning(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        v = [ctypes.c_int() for _ in range(5)]
        ms = ctypes.c_float()
        self._check(self.lib.ism_get_launch_tuning(self.h, *[ctypes.byref(x) for x in v], ctypes.byref(ms)))
        return {"seg_len": a.value, "wg_per_cu": b.value, "graphs": c.value, "interleave": v[2].value,
                "autotune": v[3].value, "tuned_buckets": v[4].value, "tuned_ms": ms.value}

    def set_autotune(self, enable=True):
        """Tune each new shape bucket on its first batch (ism_set_autotune)."""
        self._check(self.lib.ism_set_autotune(self.h, int(bool(enable))))

    # -- RIRs
    @staticmethod
    def _check_out(out, n):
        """A caller-supplied output must hold n contiguous float32 elements on the device."""
        import torch
        if out.dtype != torch.float32 or not out.is_cuda or not out.is_contiguous() or out.numel() < n:
            raise ValueError(f"out must be a contiguous CUDA float32 tensor of at least {n} elements")

    @staticmethod
    def _check_in(t, name, n=0):
        """A device input must be contiguous float32 (and hold at least n elements)."""
        import torch
        if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or t.numel() < n:
            raise ValueError(f"{name} must be a contiguous CUDA float32 tensor" + (f" of at least {n} elements" if n else ""))

    def rir(self, L, beta, src, mics, fs, c, max_order, rir_len, fd_taps,
            order_mode=ORDER_INDEX_L1, precision=PREC_FP32, out=None, stream=None):
        """One room: returns (or fills) a float32 device tensor [M, rir_len]."""
        import torch
        L = np.ascontiguousarray(L, dtype=np.float64)
        beta = np.ascontiguousarray(beta, dtype=np.float64)
        src = np.ascontiguousarray(src, dtype=np.float64)
        mics = np.ascontiguousarray(np.atleast_2d(mics), dtype=np.float64)
        M = mics.shape[0]
        if out is None:
            with _on(stream):
                out = torch.empty((M, int(rir_len)), dtype=torch.float32, device="cuda")
        else:
            self._check_out(out, M * max(int(rir_len), 0))
        rc = self.lib.ism_rir(self.h, _dptr(L), _dptr(beta), _dptr(src), int(M), _dptr(mics), float(fs),
                              float(c), int(max_order), int(order_mode), int(rir_len), int(fd_taps),
                              int(precision), ctypes.c_void_p(out.data_ptr()), _stream_handle(stream))
        self._check(rc)
        return out

    def rir_batch(self, batch, precision=PREC_FP32, out=None, stream=None, rooms=None):
        """A scene batch in one launch: returns (or fills) a flat float32 device tensor."""
        import torch
        if rooms is None:
            rooms = rooms_array(batch)
        mics = np.ascontiguousarray(batch["mics"], dtype=np.float64)
        if out is None:
            with _on(stream):
                out = torch.empty(int(batch["out_size"]), dtype=torch.float32, device="cuda")
        else:
            self._check_out(out, int(batch["out_size"]))
        rc = self.lib.ism_rir_batch(self.h, len(rooms), rooms.ctypes.data_as(ctypes.c_void_p), _dptr(mics),
                                    float(batch["fs"]), float(batch["c"]), int(batch["fd_taps"]),
                                    int(batch["order_mode"]), int(precision), ctypes.c_void_p(out.data_ptr()),
                                    _stream_handle(stream))
        self._check(rc)
        return out

    def last_counts(self):
        """(taps, records, images tested) of the last RIR call; waits for it."""
        c = (ctypes.c_int64 * 8)()
        self._check(self.lib.ism_last_counts(self.h, c))
        return {"taps": int(c[0]), "records": int(c[1]), "images": int(c[2]), "rounds": int(c[3]),
                "chunks": int(c[4]), "steps": int(c[5]), "deferred": int(c[6])}

    def plan_stats(self, batch):
        rooms = rooms_array(batch)
        mics = np.ascontiguousarray(batch["mics"], dtype=np.float64)
        n = ctypes.c_int64()
        rec, taps = ctypes.c_double(), ctypes.c_double()
        self._check(self.lib.ism_batch_plan_stats(self.h, len(rooms), rooms.ctypes.data_as(ctypes.c_void_p),
                                                  _dptr(mics), float(batch["fs"]), float(batch["c"]),
                                                  int(batch["fd_taps"]), ctypes.byref(n), ctypes.byref(rec),
                                                  ctypes.byref(taps)))
        return {"items": n.value, "est_records": rec.value, "est_taps": taps.value}

    def autotune(self, batch, candidates=None, precision=PREC_FP32, out=None, stream=None):
        import torch
        rooms = rooms_array(batch)
        mics = np.ascontiguousarray(batch["mics"], dtype=np.float64)
        if out is None:
            with _on(stream):
                out = torch.empty(int(batch["out_size"]), dtype=torch.float32, device="cuda")
        else:
            self._check_out(out, int(batch["out_size"]))
        cand = list(candidates or [])
        carr = (ctypes.c_int * max(1, len(cand)))(*cand)
        best = ctypes.c_int()
        self._check(self.lib.ism_autotune(self.h, len(rooms), rooms.ctypes.data_as(ctypes.c_void_p), _dptr(mics),
                                          float(batch["fs"]), float(batch["c"]), int(batch["fd_taps"]),
                                          int(batch["order_mode"]), int(precision),
                                          ctypes.c_void_p(out.data_ptr()), _stream_handle(stream), carr,
                                          len(cand), ctypes.byref(best)))
        return best.value

    # -- source convolution
    def convolve_batch(self, rirs, rir_offset, rir_len, M, src, out_len, snr_db=None, z=None, noise_seed=None,
                       use_mfma=True, out=None, stream=None):
        """RIRs (flat device tensor) convolved with sources [R, src_len] (device), plus sensor noise
        at snr_db (per room) when given: deviates z [R, M, out_len] from the caller
        (ism_convolve_batch_z), or drawn on the device from noise_seed (ism_convolve_batch)."""
        import torch
        R = int(src.shape[0])
        off = np.ascontiguousarray(rir_offset, dtype=np.int64)
        ln = np.ascontiguousarray(rir_len, dtype=np.int32)
        self._check_in(src, "src")
        self._check_in(rirs, "rirs", int((off + int(M) * ln.astype(np.int64)).max()) if off.size else 0)
        if snr_db is not None and (z is None) == (noise_seed is None):
            raise ValueError("with snr_db give exactly one of z (deviates) and noise_seed")
        if z is not None:
            self._check_in(z, "z", R * int(M) * max(int(out_len), 0))
        if out is None:
            with _on(stream):
                out = torch.empty((R, int(M), int(out_len)), dtype=torch.float32, device="cuda")
        else:
            self._check_out(out, R * int(M) * max(int(out_len), 0))
        snr_p = None
        if snr_db is not None:
            snr = np.ascontiguousarray(snr_db, dtype=np.float32)
            snr_p = snr.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        args = (self.h, R, int(M), ctypes.c_void_p(rirs.data_ptr()),
                off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), ln.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                ctypes.c_void_p(src.data_ptr()), int(src.shape[1]), int(out_len), snr_p)
        tail = (int(bool(use_mfma)), ctypes.c_void_p(out.data_ptr()), _stream_handle(stream))
        if z is not None:
            rc = self.lib.ism_convolve_batch_z(*args, ctypes.c_void_p(z.data_ptr()), *tail)
        else:
            rc = self.lib.ism_convolve_batch(*args, int(noise_seed or 0) & 0xFFFFFFFFFFFFFFFF, *tail)
        self._check(rc)
        return out

    def normal_deviates(self, n_rooms, M, n_samples, seed, out=None, stream=None):
        """Seeded standard normal deviates [n_rooms, M, n_samples] (float32, device): the sensor
        noise that convolve_batch draws for noise_seed = seed."""
        import torch
        if out is None:
            with _on(stream):
                out = torch.empty((int(n_rooms), int(M), int(n_samples)), dtype=torch.float32, device="cuda")
        else:
            self._check_out(out, int(n_rooms) * int(M) * int(n_samples))
        self._check(self.lib.ism_normal_deviates(self.h, int(n_rooms), int(M), int(n_samples),
                                                 int(seed) & 0xFFFFFFFFFFFFFFFF, ctypes.c_void_p(out.data_ptr()),
                                                 _stream_handle(stream)))
        return out

    def set_conv_timing(self, on):
        """Record HIP events around the kernels of each later convolve_batch call (off by default)."""
        self._check(self.lib.ism_conv_set_timing(self.h, 1 if on else 0))

    def conv_last_timing(self):
        """(pack, convolution, noise) kernel durations in ms of the last timed convolve_batch call
        (waits for it)."""
        ms = (ctypes.c_float * 3)()
        self._check(self.lib.ism_conv_last_timing(self.h, ms))
        return float(ms[0]), float(ms[1]), float(ms[2])

    # -- reverberation time
    def rir_t30(self, rir, fs, stream=None):
        """T30 (s) of a device FP32 RIR tensor (+inf if its decay does not reach -35 dB)."""
        import torch
        with _on(stream):
            rir = rir.contiguous()
            self._check_in(rir, "rir")
            t = torch.empty(1, dtype=torch.float64, device="cuda")
            self._check(self.lib.ism_rir_t30(self.h, ctypes.c_void_p(rir.data_ptr()), int(rir.numel()), float(fs),
                                             ctypes.c_void_p(t.data_ptr()), _stream_handle(stream)))
            # the copy to the host runs on the stream that wrote t
            return float(t.cpu()[0])

    def fit_beta(self, L, src, mic, fs, c, fd_taps, rt_target, rir_len, iters=30, stream=None):
        """Uniform beta whose simulated RIR (src -> mic) has T30 = rt_target.  Returns (beta, T30)."""
        import torch
        with _on(stream):
            work = torch.empty(int(self.lib.ism_rt_work_bytes(int(rir_len))), dtype=torch.uint8, device="cuda")
        L_ = np.ascontiguousarray(L, dtype=np.float64)
        s_ = np.ascontiguousarray(src, dtype=np.float64)
        m_ = np.ascontiguousarray(mic, dtype=np.float64)
        beta, rt = ctypes.c_double(), ctypes.c_double()
        self._check(self.lib.ism_fit_beta(self.h, _dptr(L_), _dptr(s_), _dptr(m_), float(fs), float(c), int(fd_taps),
                                          float(rt_target), int(rir_len), int(iters),
                                          ctypes.c_void_p(work.data_ptr()), int(work.numel()),
                                          ctypes.byref(beta), ctypes.byref(rt), _stream_handle(stream)))
        return beta.value, rt.value


    def fit_beta_mean(self, L, srcs, mics, fs, c, fd_taps, rt_target, rir_len, iters=30, stream=None):
        """Uniform beta whose RIRs from every source to every microphone have a mean T30 of
        rt_target.  Returns (beta, mean T30)."""
        import torch
        srcs = np.ascontiguousarray(np.atleast_2d(srcs), dtype=np.float64)
        mics = np.ascontiguousarray(np.atleast_2d(mics), dtype=np.float64)
        n_src, M = srcs.shape[0], mics.shape[0]
        nbytes = int(self.lib.ism_rt_mean_work_bytes(int(n_src), int(M), int(rir_len)))
        with _on(stream):
            work = torch.empty(max(nbytes, 1), dtype=torch.uint8, device="cuda")
        L_ = np.ascontiguousarray(L, dtype=np.float64)
        beta, rt = ctypes.c_double(), ctypes.c_double()
        self._check(self.lib.ism_fit_beta_mean(self.h, _dptr(L_), int(n_src), _dptr(srcs), int(M), _dptr(mics),
                                               float(fs), float(c), int(fd_taps), float(rt_target), int(rir_len),
                                               int(iters), ctypes.c_void_p(work.data_ptr()), int(work.numel()),
                                               ctypes.byref(beta), ctypes.byref(rt), _stream_handle(stream)))
        return beta.value, rt.value


SERVER_STATES = {0: "queued", 1: "running", 2: "done", 3: "failed"}


class Server:
    """Continuous-batching RIR engine (ism_server_*)."""

    def __init__(self, n_lanes=4, hbm_budget_bytes=8 << 30, max_batch_rooms=64, mock=False):
        self.lib = load()
        s = ctypes.c_void_p()
        rc = self.lib.ism_server_create(int(n_lanes), int(hbm_budget_bytes), int(max_batch_rooms), int(bool(mock)),
                                        ctypes.byref(s))
        if rc != ISM_OK:
            raise IsmError(rc, "ism_server_create failed: " + self.lib.ism_strerror(rc).decode())
        self.s = s

    def close(self):
        if getattr(self, "s", None):
            self.lib.ism_server_destroy(self.s)
            self.s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != ISM_OK:
            raise IsmError(rc, self.lib.ism_server_last_error(self.s).decode() or self.lib.ism_strerror(rc).decode())

    def submit(self, L, beta, src, mics, rir_len, fs, c, fd_taps, max_order=-1, order_mode=ORDER_INDEX_L1,
               precision=PREC_FP32):
        r = np.zeros(1, dtype=ROOM_DTYPE)
        mics = np.ascontiguousarray(np.atleast_2d(mics), dtype=np.float64)
        r["L"], r["beta"], r["src"] = L, beta, src
        r["n_mics"], r["max_order"], r["rir_len"] = mics.shape[0], max_order, rir_len
        t = ctypes.c_uint64()
        self._check(self.lib.ism_server_submit(self.s, r.ctypes.data_as(ctypes.c_void_p), _dptr(mics), float(fs),
                                               float(c), int(fd_taps), int(order_mode), int(precision),
                                               ctypes.byref(t)))
        return t.value

    def poll(self, ticket):
        st, ptr, lat = ctypes.c_int(), ctypes.c_void_p(), ctypes.c_double()
        rc = self.lib.ism_server_poll(self.s, ctypes.c_uint64(ticket), ctypes.byref(st), ctypes.byref(ptr),
                                      ctypes.byref(lat))
        if st.value != 3:
            self._check(rc)
        return SERVER_STATES[st.value], ptr.value, lat.value

    def result(self, ticket, M, rir_len, stream=None):
        """Copy a finished result into a new device tensor [M, rir_len]."""
        import torch
        with _on(stream):
            out = torch.empty((M, rir_len), dtype=torch.float32, device="cuda")
        self._check(self.lib.ism_server_copy_result(self.s, ctypes.c_uint64(ticket), ctypes.c_void_p(out.data_ptr()),
                                                    _stream_handle(stream)))
        return out

    def release(self, ticket):
        self._check(self.lib.ism_server_release(self.s, ctypes.c_uint64(ticket)))

    def stats(self):
        st = (ctypes.c_int64 * 8)()
        self._check(self.lib.ism_server_stats(self.s, st))
        keys = ["submitted", "done", "batches", "max_concurrent_batches", "pool_bytes", "pool_peak_bytes",
                "queued", "rirs_done"]
        return dict(zip(keys, [int(v) for v in st]))

    def counters(self):
        v = (ctypes.c_int64 * 8)()
        self._check(self.lib.ism_server_counters(self.s, v))
        keys = ["budget_bytes", "pool_bytes", "staging_bytes", "pool_peak_bytes", "admission_stalls", "taps_done",
                "records_done", "rirs_done"]
        return dict(zip(keys, [int(x) for x in v]))

    def replay(self, batch, arrival_s):
        """Submit the rooms of a scene batch at the given arrival times; returns (latencies ms, wall s)."""
        rooms = rooms_array(batch)
        mics = np.ascontiguousarray(batch["mics"], dtype=np.float64)
        arr = np.ascontiguousarray(arrival_s, dtype=np.float64)
        lat = np.zeros(len(rooms))
        wall = ctypes.c_double()
        rc = self.lib.ism_server_replay(self.s, len(rooms), rooms.ctypes.data_as(ctypes.c_void_p), _dptr(mics),
                                        _dptr(arr), float(batch["fs"]), float(batch["c"]), int(batch["fd_taps"]),
                                        _dptr(lat), ctypes.byref(wall))
        self._check(rc)
        return lat, wall.value
