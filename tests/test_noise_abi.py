"""C-ABI checks of the convolution / sensor-noise entry points that need no GPU: argument
validation before any device work (ISM_EINVAL), and ISM_EDEVICE, not a fallback, when the
arguments are valid but no device exists."""
import ctypes

import numpy as np
import pytest

from paper_2104_13347_amd import ism


@pytest.fixture(scope="module")
def handle():
    h = ism.Handle()
    yield h
    h.close()


def _gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.mark.parametrize("R,M,n", [(-1, 8, 16), (1, 0, 16), (1, 8, 0), (70000, 8, 16), (1, 8, (1 << 28) + 1)])
def test_normal_deviates_validation(handle, R, M, n):
    assert handle.lib.ism_normal_deviates(handle.h, R, M, n, 7, ctypes.c_void_p(4096), None) == ism.ISM_EINVAL


def test_normal_deviates_needs_output(handle):
    assert handle.lib.ism_normal_deviates(handle.h, 1, 8, 16, 7, None, None) == ism.ISM_EINVAL
    assert handle.lib.ism_normal_deviates(handle.h, 0, 8, 16, 7, None, None) == ism.ISM_OK   # nothing to do


@pytest.mark.skipif(_gpu(), reason="checks the no-device path")
def test_normal_deviates_without_device_fails_loudly(handle):
    assert handle.lib.ism_normal_deviates(handle.h, 1, 8, 16, 7, ctypes.c_void_p(4096), None) == ism.ISM_EDEVICE


def _conv(handle, n_rooms=2, M=8, lens=(10, 20), src_len=100, out_len=50, snr=(10.0, 20.0), seeded=True,
          mfma=1, z=4096):
    off = np.ascontiguousarray([0, M * lens[0]][:max(n_rooms, 0)] + [0] * max(0, n_rooms - 2), dtype=np.int64)
    ln = np.ascontiguousarray(list(lens)[:max(n_rooms, 0)] + [10] * max(0, n_rooms - 2), dtype=np.int32)
    sn = np.ascontiguousarray(list(snr)[:max(n_rooms, 0)] + [10.0] * max(0, n_rooms - 2), dtype=np.float32)
    P = lambda a, t: a.ctypes.data_as(ctypes.POINTER(t))
    args = (handle.h, n_rooms, M, ctypes.c_void_p(4096), P(off, ctypes.c_int64), P(ln, ctypes.c_int32),
            ctypes.c_void_p(4096), src_len, out_len, P(sn, ctypes.c_float) if snr is not None else None)
    if seeded:
        return handle.lib.ism_convolve_batch(*args, 1234, mfma, ctypes.c_void_p(4096), None)
    return handle.lib.ism_convolve_batch_z(*args, ctypes.c_void_p(z) if z else None, mfma, ctypes.c_void_p(4096),
                                           None)


@pytest.mark.parametrize("kw", [dict(M=0), dict(src_len=0), dict(out_len=0), dict(n_rooms=70000),
                                dict(M=4), dict(lens=(0, 20)), dict(snr=(float("nan"), 1.0)),
                                dict(seeded=False, z=0)])
def test_convolve_validation(handle, kw):
    # MFMA path with 4 microphones, an empty RIR, a non-finite SNR, noise without deviates
    assert _conv(handle, **kw) == ism.ISM_EINVAL


@pytest.mark.skipif(_gpu(), reason="checks the no-device path")
def test_convolve_without_device_fails_loudly(handle):
    assert _conv(handle) == ism.ISM_EDEVICE


def test_conv_timing_needs_a_timed_call():
    # a fresh handle: nothing timed yet; switching timing on touches no device
    h = ism.Handle()
    try:
        ms = (ctypes.c_float * 3)()
        assert h.lib.ism_conv_last_timing(h.h, ms) == ism.ISM_EINVAL
        assert h.lib.ism_conv_last_timing(h.h, None) == ism.ISM_EINVAL
        assert h.lib.ism_conv_set_timing(None, 1) == ism.ISM_EINVAL
        assert h.lib.ism_conv_set_timing(h.h, 1) == ism.ISM_OK
        assert h.lib.ism_conv_last_timing(h.h, ms) == ism.ISM_EINVAL
        assert h.lib.ism_conv_set_timing(h.h, 0) == ism.ISM_OK
    finally:
        h.close()
