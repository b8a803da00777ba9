"""C-ABI checks that need no GPU: the library loads, exports every function
include/ism.h declares, validates arguments before any device work (each
error code), plans batches exactly, and fails loudly without a device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2104_13347_amd import ism, scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ism.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ism_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = ism.load()
    names = _declared()
    assert "ism_rir" in names and "ism_rir_batch" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(ism.EXPORTS) <= set(names)
    assert lib.ism_version() == 100


def test_room_struct_layout_matches_header():
    assert ism.ROOM_DTYPE.itemsize == 120
    assert ism.ROOM_DTYPE.fields["out_offset"][1] == 112


@pytest.fixture(scope="module")
def handle():
    h = ism.Handle()
    yield h
    h.close()


def _call(h, **kw):
    a = dict(L=[5.0, 4.0, 3.0], beta=[0.7] * 6, src=[1.3, 2.1, 1.5], mics=[[3.6, 1.7, 1.2]], fs=16000.0,
             c=343.0, max_order=10, order_mode=0, rir_len=64, fd_taps=9, precision=0)
    a.update(kw)
    L = np.asarray(a["L"], dtype=np.float64)
    beta = np.asarray(a["beta"], dtype=np.float64)
    src = np.asarray(a["src"], dtype=np.float64)
    mics = np.ascontiguousarray(np.atleast_2d(a["mics"]), dtype=np.float64)
    P = lambda x: x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    out = ctypes.c_void_p(0 if a.get("null_out") else 0x1000)   # never dereferenced: validation fails first
    return h.lib.ism_rir(h.h, P(L), P(beta), P(src), int(mics.shape[0]), P(mics), float(a["fs"]), float(a["c"]),
                         int(a["max_order"]), int(a["order_mode"]), int(a["rir_len"]), int(a["fd_taps"]),
                         int(a["precision"]), out, ctypes.c_void_p(0))


@pytest.mark.parametrize("kw,code", [
    (dict(fd_taps=6), ism.ISM_EINVAL),
    (dict(fd_taps=8, precision=4), ism.ISM_EINVAL),
    (dict(fd_taps=0), ism.ISM_EINVAL),
    (dict(fd_taps=257), ism.ISM_EINVAL),
    (dict(rir_len=0), ism.ISM_EINVAL),
    (dict(fs=0.0), ism.ISM_EINVAL),
    (dict(c=float("nan")), ism.ISM_EINVAL),
    (dict(L=[5.0, -4.0, 3.0]), ism.ISM_EINVAL),
    (dict(beta=[0.7] * 5 + [1.5]), ism.ISM_EINVAL),
    (dict(beta=[0.7] * 5 + [-0.1]), ism.ISM_EINVAL),
    (dict(order_mode=2), ism.ISM_EINVAL),
    (dict(precision=9), ism.ISM_EINVAL),
    (dict(mics=np.zeros((0, 3))), ism.ISM_EINVAL),
    (dict(null_out=True), ism.ISM_EINVAL),
    (dict(src=[0.0, 2.1, 1.5]), ism.ISM_EDOMAIN),
    (dict(src=[5.0, 2.1, 1.5]), ism.ISM_EDOMAIN),
    (dict(mics=[[3.6, 4.1, 1.2]]), ism.ISM_EDOMAIN),
    (dict(mics=[[1.3, 2.1, 1.5]]), ism.ISM_EDOMAIN),
    (dict(mics=[[float("inf"), 2.0, 1.0]]), ism.ISM_EINVAL),
])
def test_validation_error_codes(handle, kw, code):
    assert _call(handle, **kw) == code
    assert handle.lib.ism_last_error(handle.h).decode() != ""


def test_mic_on_wall_is_accepted_by_validation(handle):
    # microphones may sit on a wall (closed interval); without a GPU the call then fails on the
    # device, with a GPU it succeeds -- either way not a validation error
    rc = _call(handle, mics=[[5.0, 0.0, 3.0]])
    assert rc not in (ism.ISM_EINVAL, ism.ISM_EDOMAIN)


def test_tuning_limits(handle):
    with pytest.raises(ism.IsmError):
        handle.set_tuning(seg_len=100)
    with pytest.raises(ism.IsmError):
        handle.set_tuning(seg_len=4096)
    with pytest.raises(ism.IsmError):
        handle.set_tuning(wg_per_cu=100)
    handle.set_tuning(seg_len=512, wg_per_cu=4)
    assert handle.get_tuning()["seg_len"] == 512 and handle.get_tuning()["wg_per_cu"] == 4
    handle.set_tuning(seg_len=1024, wg_per_cu=0)


def test_plan_item_count_is_exact(handle):
    b = scenes.c1(n_rooms=12)
    handle.set_tuning(seg_len=512)
    st = handle.plan_stats(b)
    want = int(sum(m * -(-L // 512) for m, L in zip(b["n_mics"], b["rir_len"])))
    assert st["items"] == want
    # expected taps of the plan: same order as the volume law of the image count
    assert st["est_taps"] > 0
    handle.set_tuning(seg_len=1024)


def test_no_device_fails_loudly(handle):
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except Exception:
        pass
    rc = _call(handle)
    assert rc == ism.ISM_EDEVICE
    assert "device" in handle.lib.ism_last_error(handle.h).decode()


def test_paper_room_scene_geometry():
    b = scenes.paper_room1(n_sources=2000, seed=5)
    c = np.array([4.0, 6.0, 1.5])
    r = np.linalg.norm(b["src"] - c, axis=1)
    assert r.min() >= 1.5 and r.max() <= 2.5
    elev = np.degrees(np.arcsin((b["src"][:, 2] - c[2]) / r))
    assert np.abs(elev).max() <= 7.0 + 1e-9
    # uniform in volume: the median radius solves r^3 = ((1.5^3 + 2.5^3) / 2)
    assert abs(np.median(r) - ((1.5 ** 3 + 2.5 ** 3) / 2) ** (1 / 3)) < 0.03
    m = b["mics"][:7]
    assert np.allclose(m[0], c)
    assert np.allclose(np.linalg.norm(m[1:] - c, axis=1), 0.04)
    assert b["rir_len"][0] == 8000 and b["fd_taps"] == 8 and len(b["rir_len"]) == 2000


def test_second_paper_room_scene_geometry():
    # 5 x 5 x 4 m, the array centred at (2.5, 2.5, 1.5) m, the torus of radius 2 +- 0.5 m and
    # +-7 degrees, positions at least 0.1 m from every wall (the torus reaches them on the axes)
    b = scenes.paper_room2(n_sources=3000, seed=6)
    L, c = np.array([5.0, 5.0, 4.0]), np.array([2.5, 2.5, 1.5])
    src = b["src"]
    assert len(src) == 3000 and np.allclose(b["L"], L)
    assert np.all(src > 0.1) and np.all(src < L - 0.1)
    r = np.linalg.norm(src - c, axis=1)
    assert r.min() >= 1.5 and r.max() <= 2.5
    elev = np.degrees(np.arcsin((src[:, 2] - c[2]) / r))
    assert np.abs(elev).max() <= 7.0 + 1e-9
    assert np.allclose(b["mics"][0], c) and b["n_mics"][0] == 7
    assert b["rir_len"][0] == 8000 and b["fd_taps"] == 8
    # Sabine's coefficient for RT 0.5 s unless a fitted one is passed
    assert 0.8 < b["beta"][0][0] < 0.9
    assert scenes.paper_room2(n_sources=1, beta=0.8)["beta"][0][0] == 0.8


def test_room_too_small_for_its_rir_length_is_rejected(handle):
    # image columns past the kernels' 32-bit indexing: a 1 cm room with a 10 s RIR
    assert _call(handle, L=[0.01, 0.01, 0.01], src=[0.005, 0.005, 0.005], mics=[[0.002, 0.002, 0.002]],
                 rir_len=160000, max_order=-1) == ism.ISM_EINVAL
    assert "too many images" in handle.lib.ism_last_error(handle.h).decode()
