"""GPU parity of the BeamLearning forward pass (paper section II.B) against the
FP64 oracle, through the C-ABI (include/beamlearning.h).

Tolerance.  Layers 1..17 multiply FP16 pairs on the matrix cores: each
operand keeps 22 significant bits (2^-22 relative), the dropped lo*lo term is
below 2^-22 of a product and the FP32 sums over K = 384 add about
sqrt(384) 2^-24 of the summed magnitudes, so a layer's pre-norm output carries
about 1e-6 of sum |W x|.  The layer norm divides by the map's standard
deviation (a few times smaller than sum |W x| for these weights), tanh does not
amplify, and 17 residual layers add their errors.  The head's layer norm
divides the pseudo-energies by their spread across the 128 channels.  The
bound used here, ATOL + RTOL |ref| on the 128 features and the outputs, keeps
a margin of about 10x over the largest error measured on these cases.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import beamlearning as ref
from paper_2104_13347_amd import beamlearning as blm
from paper_2104_13347_amd import bl_data, ism

ATOL = 2e-5
RTOL = 1e-5


@pytest.fixture(scope="module")
def handle():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    h = ism.Handle()
    yield h
    h.close()


def _model(handle, seed, c_in=7, n_out=2, mode=blm.REGRESSION, unit_gain=True, eps=1e-6):
    p = bl_data.make_params(seed, c_in=c_in, n_out=n_out, unit_gain=unit_gain)
    return p, blm.Model(handle, bl_data.flatten(p, c_in, n_out), c_in=c_in, n_out=n_out, mode=mode, ln_eps=eps)


def _check(tag, got_f, got_o, ref_f, ref_o):
    ef = np.abs(got_f - ref_f).max()
    eo = np.abs(got_o - ref_o).max()
    print(f"[{tag}] max |features err| {ef:.3e}  max |out err| {eo:.3e}  |f| {np.abs(ref_f).max():.3f}", flush=True)
    assert np.all(np.isfinite(got_f)) and np.all(np.isfinite(got_o))
    assert np.all(np.abs(got_f - ref_f) <= ATOL + RTOL * np.abs(ref_f)), tag
    assert np.all(np.abs(got_o - ref_o) <= ATOL + RTOL * np.abs(ref_o)), tag


@pytest.mark.parametrize("c_in,n_t,batch,n_out,mode,seed", [
    (7, 1024, 3, 2, blm.REGRESSION, 1),          # the paper's frame: 7 channels, 1024 samples
    (7, 379, 2, 2, blm.REGRESSION, 2),           # shortest frame: one valid sample
    (3, 700, 2, 37, blm.CLASSIFICATION, 3),      # ragged last tile
    (1, 1300, 1, 1, blm.REGRESSION, 4),          # one channel, 11 tiles, ragged
    (32, 520, 2, 1024, blm.CLASSIFICATION, 5),   # widest input and output
    (2, 4500, 1, 3, blm.REGRESSION, 6),          # 71 tiles: statistics over more than 64 partials
    (4, 800, 2, 16, blm.CLASSIFICATION, 7),      # largest head whose dot products span all threads
    (5, 600, 1, 17, blm.CLASSIFICATION, 8),      # smallest head with one thread per output
])
def test_forward_matches_oracle(handle, c_in, n_t, batch, n_out, mode, seed):
    p, m = _model(handle, seed, c_in=c_in, n_out=n_out, mode=mode)
    x = bl_data.frames(100 + seed, batch, c_in=c_in, n_t=n_t)
    f, o = m.forward(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    rf, ro = ref.forward(x, p, eps=1e-6, mode=mode)
    _check(f"c_in={c_in} n_t={n_t} n_out={n_out} mode={mode}", f.cpu().numpy(), o.cpu().numpy(), rf, ro)
    m.close()


def test_paper_initialisation_and_input_scales(handle):
    # gains drawn as the paper draws every variable (small), and inputs of
    # very different amplitude (layer 0 runs in FP32 on the vector units)
    p, m = _model(handle, 21, unit_gain=False)
    x = np.concatenate([bl_data.frames(22, 1, scale=1e-3), bl_data.frames(23, 1, scale=300.0)])
    f, o = m.forward(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    rf, ro = ref.forward(x, p, eps=1e-6)
    _check("paper init, scales 1e-3 / 300", f.cpu().numpy(), o.cpu().numpy(), rf, ro)
    m.close()


def test_offsets_and_strides_read_frames_in_place(handle):
    # frames cut from longer multichannel recordings (room x mic x sample), as
    # the convolution stage lays them out: per-frame offsets, channel stride
    p, m = _model(handle, 31)
    rng = np.random.default_rng(32)
    rec = rng.standard_normal((3, 8, 5000)).astype(np.float32)
    starts = [(0, 0), (0, 1024), (1, 3000), (2, 3976)]
    offs = np.array([r * 8 * 5000 + s for r, s in starts], dtype=np.int64)
    d = torch.from_numpy(rec).cuda()
    f, o = m.forward(d, n_t=1024, batch=len(starts), offsets=torch.from_numpy(offs).cuda(), ch_stride=5000)
    torch.cuda.synchronize()
    x = np.stack([rec[r, :7, s:s + 1024] for r, s in starts])
    rf, ro = ref.forward(x, p, eps=1e-6)
    _check("offsets", f.cpu().numpy(), o.cpu().numpy(), rf, ro)
    # the same frames as a contiguous batch give bitwise the same result
    f2, o2 = m.forward(torch.from_numpy(np.ascontiguousarray(x)).cuda())
    torch.cuda.synchronize()
    assert torch.equal(f, f2) and torch.equal(o, o2)
    m.close()


def test_batch_invariance_and_repeatability(handle):
    p, m = _model(handle, 41)
    x = torch.from_numpy(bl_data.frames(42, 6)).cuda()
    f, o = m.forward(x)
    f1, o1 = m.forward(x[2:3])
    fr, orr = m.forward(x)
    torch.cuda.synchronize()
    assert torch.equal(f[2:3], f1) and torch.equal(o[2:3], o1)
    assert torch.equal(f, fr) and torch.equal(o, orr)
    assert m.forward(x[:0])[1].shape == (0, 2)
    m.close()


@pytest.mark.parametrize("batch", [4, 6, 12])
def test_every_tile_height_equals_single_frames(handle, batch):
    # frames of 1000 samples on 256 CUs: a frame alone and a batch of 4 run layers 1..17
    # in 16-row tiles, a batch of 6 in 32-row tiles and a batch of 12 in 64-row tiles
    # (low-latency form); the layer-norm partials are per 16 rows in every form, so each
    # frame's result is bitwise the same as when it runs alone
    p, m = _model(handle, 81 + batch)
    x = torch.from_numpy(bl_data.frames(90 + batch, batch, n_t=1000)).cuda()
    f, o = m.forward(x)
    singles = [m.forward(x[i:i + 1]) for i in range(batch)]
    torch.cuda.synchronize()
    assert torch.equal(f, torch.cat([s[0] for s in singles]))
    assert torch.equal(o, torch.cat([s[1] for s in singles]))
    rf, ro = ref.forward(x[-1:].cpu().numpy(), p, eps=1e-6)
    _check(f"batch {batch} x 1000, last frame", f[-1:].cpu().numpy(), o[-1:].cpu().numpy(), rf, ro)
    m.close()


@pytest.mark.parametrize("batch", [40, 50])
def test_shortest_frames_in_64_row_tiles_equal_single_frames(handle, batch):
    # frames of 379 samples (one valid output sample; the last 64-row tile holds 59 rows)
    # on 256 CUs: a batch of 40 runs 64-row tiles in the low-latency form, a batch of 50
    # at full occupancy; each frame alone runs 16-row tiles
    p, m = _model(handle, 101 + batch)
    x = torch.from_numpy(bl_data.frames(110 + batch, batch, n_t=379)).cuda()
    f, o = m.forward(x)
    singles = [m.forward(x[i:i + 1]) for i in range(batch)]
    torch.cuda.synchronize()
    assert torch.equal(f, torch.cat([s[0] for s in singles]))
    assert torch.equal(o, torch.cat([s[1] for s in singles]))
    rf, ro = ref.forward(x[:1].cpu().numpy(), p, eps=1e-6)
    _check(f"batch {batch} x 379, first frame", f[:1].cpu().numpy(), o[:1].cpu().numpy(), rf, ro)
    m.close()


def test_full_batch_sampled(handle):
    # the benchmark's launch: 3600 frames of 7 x 1024 in one call; frames
    # sampled across the batch are checked against the oracle one by one
    p, m = _model(handle, 51, unit_gain=False)
    B = 3600
    x = torch.randn((B, 7, 1024), generator=torch.Generator().manual_seed(52)).cuda()
    f, o = m.forward(x)
    torch.cuda.synchronize()
    idx = [0, 1799, 3599]
    xs = x[idx].cpu().numpy()
    rf, ro = ref.forward(xs, p, eps=1e-6)
    _check("3600 frames, sampled", f[idx].cpu().numpy(), o[idx].cpu().numpy(), rf, ro)
    assert torch.isfinite(o).all()
    m.close()


def test_invalid_arguments(handle):
    p, m = _model(handle, 61)
    x = torch.zeros((1, 7, 378), device="cuda")
    with pytest.raises(ism.IsmError):
        m.forward(x)                                   # shorter than the receptive field
    x = torch.zeros((2, 7, 1024), device="cuda")
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(ism.IsmError):
        m.forward(x, workspace=ws)                     # workspace too small
    with pytest.raises(ValueError):
        blm.Model(handle, np.zeros(10, np.float32))
    with pytest.raises(ValueError):
        m.forward(x, out=torch.empty((1, 2), device="cuda"))                     # too small for 2 frames
    with pytest.raises(ValueError):
        m.forward(x, out=torch.empty((2, 2), dtype=torch.float64, device="cuda"))  # wrong type
    with pytest.raises(ValueError):
        m.forward(x.double())                                                    # frames of another type
    m.close()


def test_large_ragged_batch_equals_single_frames(handle):
    # 64 frames of 1000 samples (1024 tiles, the last of each frame ragged) in one call
    # equal each frame run alone, bitwise; sampled frames against the oracle
    p, m = _model(handle, 71)
    x = bl_data.frames(72, 64, n_t=1000)
    xd = torch.from_numpy(x).cuda()
    f, o = m.forward(xd)
    singles = [m.forward(xd[i:i + 1]) for i in range(64)]
    torch.cuda.synchronize()
    assert torch.equal(f, torch.cat([s[0] for s in singles]))
    assert torch.equal(o, torch.cat([s[1] for s in singles]))
    idx = [0, 33, 63]
    rf, ro = ref.forward(x[idx], p, eps=1e-6)
    _check("64 x 1000, sampled", f[idx].cpu().numpy(), o[idx].cpu().numpy(), rf, ro)
    m.close()


def test_slices_of_one_offsets_tensor(handle):
    # windows of one device offsets tensor (offsets[:b], offsets[i:i+1], as a serving loop
    # passes them on every call) give the frames a fresh tensor of the same values gives,
    # and a window that reaches past x is still refused after the others passed
    p, m = _model(handle, 51)
    rng = np.random.default_rng(52)
    rec = rng.standard_normal((2, 8, 3000)).astype(np.float32)
    offs = np.array([0, 1500, 8 * 3000 + 700, 8 * 3000 + 1976], dtype=np.int64)
    d = torch.from_numpy(rec).cuda()
    od = torch.from_numpy(offs).cuda()
    for lo, hi in [(0, 1), (0, 4), (2, 3), (0, 1), (1, 4)]:
        f, o = m.forward(d, n_t=1024, batch=hi - lo, offsets=od[lo:hi], ch_stride=3000)
        f2, o2 = m.forward(d, n_t=1024, batch=hi - lo, offsets=torch.from_numpy(offs[lo:hi].copy()).cuda(),
                           ch_stride=3000)
        torch.cuda.synchronize()
        assert torch.equal(f, f2) and torch.equal(o, o2), (lo, hi)
    # in place: frame 3 now ends at 29000 + 6 x 3000 + 1024 = 48024, past the 48000 of x
    od[3:].fill_(29000)
    with pytest.raises(ValueError):
        m.forward(d, n_t=1024, batch=1, offsets=od[3:], ch_stride=3000)
    m.close()


def test_explicit_layout_is_checked_before_launch(handle):
    # an explicit frame layout that would read past x, or leaves a stride or the frame
    # count open, is refused on the host (the kernels cannot check device offsets)
    p, m = _model(handle, 41, c_in=3, n_out=2)
    x = torch.zeros(3 * 1000, device="cuda")
    with pytest.raises(ValueError):          # ch_stride missing
        m.forward(x, n_t=1000, batch=1, ex_stride=3000)
    with pytest.raises(ValueError):          # neither offsets nor ex_stride
        m.forward(x, n_t=1000, batch=1, ch_stride=1000)
    with pytest.raises(ValueError):          # second frame past the end
        m.forward(x, n_t=1000, batch=2, ex_stride=3000, ch_stride=1000)
    with pytest.raises(ValueError):          # fewer offsets than frames
        m.forward(x, n_t=1000, batch=2, offsets=torch.zeros(1, dtype=torch.int64, device="cuda"), ch_stride=1000)
    with pytest.raises(ValueError):          # an offset past the end
        m.forward(x, n_t=1000, batch=1, offsets=torch.tensor([1], dtype=torch.int64, device="cuda"), ch_stride=1000)
    with pytest.raises(ValueError):          # a negative offset
        m.forward(x, n_t=500, batch=1, offsets=torch.tensor([-1], dtype=torch.int64, device="cuda"), ch_stride=1000)
    # exactly the extent of x is accepted
    f, o = m.forward(x, n_t=1000, batch=1, ex_stride=3000, ch_stride=1000)
    torch.cuda.synchronize()
    assert torch.isfinite(o).all()
    m.close()


def test_side_stream_equals_default_stream(handle):
    # a forward pass and a T30 queued on a non-current stream give the default-stream
    # results: temporaries are allocated and written on that stream and t30 is read after it
    p, m = _model(handle, 43, c_in=7, n_out=2)
    x = torch.from_numpy(bl_data.frames(44, 5, n_t=900)).cuda()
    f0, o0 = m.forward(x)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    f1, o1 = m.forward(x, stream=s)
    s.synchronize()
    assert torch.equal(f0, f1) and torch.equal(o0, o1)
    m.close()
    rir = handle.rir([4.0, 5.0, 3.0], [0.8] * 6, [1.2, 1.5, 1.4], [[2.9, 3.6, 1.6]], 8000.0, 343.0, -1, 4000, 9)[0]
    torch.cuda.synchronize()
    t_def = handle.rir_t30(rir, 8000.0)
    s.wait_stream(torch.cuda.current_stream())
    t_side = handle.rir_t30(rir[::1], 8000.0, stream=s)
    assert t_def == t_side and math.isfinite(t_def)
