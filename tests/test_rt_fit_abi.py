"""C-ABI checks of the reverberation-time entry points that need no GPU: work
size and argument validation before any device work."""
import ctypes

import numpy as np
import pytest

from paper_2104_13347_amd import ism


@pytest.fixture(scope="module")
def handle():
    h = ism.Handle()
    yield h
    h.close()


def test_work_bytes():
    lib = ism.load()
    assert lib.ism_rt_work_bytes(0) == 0
    assert lib.ism_rt_work_bytes(16000) >= 16000 * 4 + 8


@pytest.mark.parametrize("kw", [dict(rt=0.0), dict(rt=float("nan")), dict(iters=0), dict(iters=61),
                                dict(work_bytes=16), dict(rir_len=0)])
def test_fit_beta_validation(handle, kw):
    lib = ism.load()
    d = lambda v: np.ascontiguousarray(v, dtype=np.float64)
    L, s, m = d([4.0, 5.0, 3.0]), d([1.2, 1.5, 1.4]), d([2.9, 3.6, 1.6])
    p = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    beta, rt = ctypes.c_double(), ctypes.c_double()
    rc = lib.ism_fit_beta(handle.h, p(L), p(s), p(m), 8000.0, 343.0, 8, kw.get("rt", 0.25), kw.get("rir_len", 5000),
                          kw.get("iters", 20), ctypes.c_void_p(4096), kw.get("work_bytes", 1 << 20),
                          ctypes.byref(beta), ctypes.byref(rt), None)
    assert rc == ism.ISM_EINVAL
    assert handle.lib.ism_last_error(handle.h).decode() != ""


def test_rir_t30_validation(handle):
    lib = ism.load()
    assert lib.ism_rir_t30(handle.h, None, 100, 8000.0, ctypes.c_void_p(4096), None) == ism.ISM_EINVAL
    assert lib.ism_rir_t30(handle.h, ctypes.c_void_p(4096), 100, 0.0, ctypes.c_void_p(4096), None) == ism.ISM_EINVAL


@pytest.mark.parametrize("kw", [dict(rt=0.0), dict(iters=0), dict(n_src=0), dict(M=0), dict(work_bytes=16),
                                dict(rir_len=0), dict(n_src=300, M=300)])
def test_fit_beta_mean_validation(handle, kw):
    # every malformed argument is refused before any device work (ISM_EINVAL), also without a GPU
    lib = ism.load()
    n_src, M = kw.get("n_src", 2), kw.get("M", 3)
    d = lambda v: np.ascontiguousarray(v, dtype=np.float64)
    L = d([4.0, 5.0, 3.0])
    srcs = d(np.tile([1.2, 1.5, 1.4], (max(n_src, 1), 1)))
    mics = d(np.tile([2.9, 3.6, 1.6], (max(M, 1), 1)))
    p = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    beta, rt = ctypes.c_double(), ctypes.c_double()
    rc = lib.ism_fit_beta_mean(handle.h, p(L), n_src, p(srcs), M, p(mics), 8000.0, 343.0, 8, kw.get("rt", 0.25),
                               kw.get("rir_len", 5000), kw.get("iters", 20), ctypes.c_void_p(4096),
                               kw.get("work_bytes", 1 << 30), ctypes.byref(beta), ctypes.byref(rt), None)
    assert rc == ism.ISM_EINVAL


def test_mean_work_bytes():
    lib = ism.load()
    assert lib.ism_rt_mean_work_bytes(0, 7, 100) == 0
    assert lib.ism_rt_mean_work_bytes(8, 7, 16000) >= 8 * 7 * (16000 * 4 + 8)
