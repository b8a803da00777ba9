"""C-ABI checks of the BeamLearning entry points that need no GPU: exports,
the parameter count of the documented layout, workspace sizes and argument
validation before any device work."""
import ctypes
import os
import re

import pytest

from paper_2104_13347_amd import beamlearning as blm
from paper_2104_13347_amd import bl_data, ism

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "beamlearning.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bl_[a-z_0-9]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    lib = blm.load()
    names = _declared()
    assert set(names) == set(blm.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


@pytest.mark.parametrize("c_in,n_out", [(7, 2), (1, 1), (32, 1024), (3, 37)])
def test_param_count_matches_layout(c_in, n_out):
    assert blm.param_count(c_in, n_out) == bl_data.param_count(c_in, n_out)


@pytest.mark.parametrize("c_in,n_out", [(0, 2), (33, 2), (7, 0), (7, 1025)])
def test_param_count_out_of_range(c_in, n_out):
    assert blm.param_count(c_in, n_out) == 0


def test_workspace_bytes():
    assert blm.workspace_bytes(1, 378) == 0          # shorter than the receptive field
    assert blm.workspace_bytes(1, (1 << 20) + 1) == 0
    a = blm.workspace_bytes(1, 1024)
    # four 128-channel FP32 maps per frame dominate
    assert a >= 4 * 1024 * 128 * 4
    assert blm.workspace_bytes(100, 1024) >= 100 * 4 * 1024 * 128 * 4
    assert blm.workspace_bytes(0, 1024) >= 0


@pytest.fixture(scope="module")
def handle():
    h = ism.Handle()
    yield h
    h.close()


@pytest.mark.parametrize("kw", [dict(c_in=0), dict(c_in=33), dict(n_out=0), dict(n_out=1025), dict(mode=2),
                                dict(eps=0.0), dict(eps=float("nan")), dict(null_params=True)])
def test_model_create_validation(handle, kw):
    lib = blm.load()
    m = ctypes.c_void_p()
    params = ctypes.c_void_p(0 if kw.get("null_params") else 4096)   # never dereferenced: rejected first
    rc = lib.bl_model_create(handle.h, kw.get("c_in", 7), kw.get("n_out", 2), kw.get("mode", 0),
                             kw.get("eps", 1e-6), params, None, ctypes.byref(m))
    assert rc == ism.ISM_EINVAL
    assert m.value is None
    assert handle.lib.ism_last_error(handle.h).decode() != ""


def test_forward_validation(handle):
    lib = blm.load()
    vp = ctypes.c_void_p
    rc = lib.bl_forward(handle.h, None, 1, 1024, vp(4096), None, 0, 0, vp(4096), 1 << 30, None, vp(4096), None)
    assert rc == ism.ISM_EINVAL and "model" in handle.lib.ism_last_error(handle.h).decode()


def test_offset_check_is_per_tensor_object():
    # the host check of an explicit frame layout reads the offsets again for every new
    # offsets tensor, even one at the address of a freed tensor that passed, and after an
    # in-place change of the same tensor (CPU tensors stand in for device ones: the check
    # only reads them)
    import types
    import torch
    fake = types.SimpleNamespace(c_in=3)
    x = torch.zeros(3 * 1000)
    check = lambda off, n_t=1000: blm.Model._check_extent(fake, x, n_t, 1, off, None, 1000)
    ok = torch.tensor([0], dtype=torch.int64)
    check(ok)
    with pytest.raises(ValueError):
        check(torch.tensor([1], dtype=torch.int64))
    for _ in range(4):      # fresh tensors, often at a reused address
        good = torch.tensor([0], dtype=torch.int64)
        check(good, n_t=500)
        del good
        with pytest.raises(ValueError):
            check(torch.tensor([-1], dtype=torch.int64), n_t=500)
    ok.fill_(1)             # in place: torch's version counter moves
    with pytest.raises(ValueError):
        check(ok)
    # a new tensor object at the very address of one that passed, with the same version
    # counter (0) but other contents
    import numpy as np
    buf = np.zeros(1, dtype=np.int64)
    t1 = torch.from_numpy(buf)
    check(t1, n_t=500)
    buf[0] = -1
    t2 = torch.from_numpy(buf)
    assert t2.data_ptr() == t1.data_ptr() and t2._version == t1._version
    with pytest.raises(ValueError):
        check(t2, n_t=500)


def test_offset_check_reuses_its_read_for_slices_of_one_tensor():
    # offsets[:b] is a new view object on every call; the check reads its values once per
    # base tensor, element offset, batch and version, so a fresh slice of unchanged offsets
    # costs no read, while another window of the base or an in-place change is read again
    import types
    import torch
    fake = types.SimpleNamespace(c_in=3)
    x = torch.zeros(3 * 1000)
    check = lambda off, n_t=500: blm.Model._check_extent(fake, x, n_t, 1, off, None, 1000)
    base = torch.tensor([0, -1, 0], dtype=torch.int64)
    check(base[:1])
    first = fake._off_range
    check(base[:1])
    assert fake._off_range is first                 # cache hit: nothing read back
    with pytest.raises(ValueError):
        check(base[1:])                             # another window of the same storage
    check(base[2:])
    assert fake._off_range is not first
    base[:1].fill_(-1)                              # in place through a view: shared version moves
    with pytest.raises(ValueError):
        check(base[:1])
