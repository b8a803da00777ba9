"""The BeamLearning forward pass without allocation (bl_forward_noalloc, the library's
fixed per-GPU workspace) against bl_forward with a caller workspace, through the C-ABI:
two calls in a row, the second with a smaller input, and a batch larger than the fixed
workspace holds at once (several passes through it).  Results equal bitwise: the same
kernels run, and a frame's result does not depend on the batch it runs in."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2104_13347_amd import beamlearning as blm
from paper_2104_13347_amd import bl_data, ism


@pytest.fixture(scope="module")
def handle():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    h = ism.Handle()
    yield h
    h.close()


def _model(h, seed, c_in=7, n_out=2):
    p = bl_data.make_params(seed, c_in=c_in, n_out=n_out)
    return blm.Model(h, bl_data.flatten(p, c_in, n_out), c_in=c_in, n_out=n_out)


def _both(m, x, **kw):
    f1, o1 = m.forward(x, **kw)
    f2, o2 = m.forward(x, noalloc=True, **kw)
    torch.cuda.synchronize()
    return (f1, o1), (f2, o2)


def test_noalloc_equals_workspace_form_twice_then_smaller(handle):
    m = _model(handle, 5)
    try:
        x = torch.from_numpy(bl_data.frames(11, 6, n_t=1024)).cuda()
        (f1, o1), (f2, o2) = _both(m, x)
        assert torch.equal(f1, f2) and torch.equal(o1, o2)
        xs = torch.from_numpy(bl_data.frames(12, 2, n_t=500)).cuda()     # second call: smaller input
        (f1, o1), (f2, o2) = _both(m, xs)
        assert torch.equal(f1, f2) and torch.equal(o1, o2)
        assert torch.isfinite(o2).all()
    finally:
        m.close()


def test_noalloc_batch_larger_than_the_fixed_workspace(handle):
    # 40 frames of 1024 samples need about 80 MiB of workspace: two passes through 64 MiB
    m = _model(handle, 6)
    try:
        assert blm.workspace_bytes(40, 1024) > handle.lib.bl_noalloc_scratch_bytes()
        x = torch.from_numpy(bl_data.frames(13, 40, n_t=1024)).cuda()
        (f1, o1), (f2, o2) = _both(m, x, features=True)
        assert torch.equal(f1, f2) and torch.equal(o1, o2)
        # explicit layout with offsets, as the benchmark cuts frames out of recordings
        flat = x.reshape(-1)
        offs = torch.arange(40, dtype=torch.int64, device="cuda") * (7 * 1024)
        (g1, p1), (g2, p2) = _both(m, flat, n_t=1024, batch=40, offsets=offs, ch_stride=1024)
        assert torch.equal(p1, p2) and torch.equal(p1, o1)
    finally:
        m.close()


def test_noalloc_refuses_a_frame_larger_than_the_workspace(handle):
    m = _model(handle, 7, c_in=1)
    try:
        x = torch.zeros(40000, device="cuda")
        with pytest.raises(ism.IsmError) as e:
            m.forward(x, n_t=40000, batch=1, ex_stride=40000, ch_stride=40000, noalloc=True)
        assert e.value.code == ism.ISM_EINVAL
    finally:
        m.close()
