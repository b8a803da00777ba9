"""GPU parity of the source convolution + sensor noise (paper section III.A)
against the FP64 oracle.  RIR inputs are seeded synthetic decaying-noise
arrays (not outputs of the GPU path).  Bars: BF16 MFMA path relative RMS error
<= 1e-2 per room; FP32 direct path max |err| <= 1e-5 x peak per room."""
import sys

import numpy as np
import pytest

import oracle
from paper_2104_13347_amd import ism, scenes

pytestmark = pytest.mark.gpu

TOL_BF16_RMS = 1e-2
TOL_FP32 = 1e-5


@pytest.fixture(scope="module")
def H():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    h = ism.Handle()
    yield h
    h.close()


def _run(H, rirs, offs, lens, x, out_len, snr=None, z=None, mfma=True):
    import torch
    M = 8
    d_rirs = torch.from_numpy(rirs).cuda()
    d_x = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    d_z = torch.from_numpy(np.ascontiguousarray(z, dtype=np.float32)).cuda() if z is not None else None
    y = H.convolve_batch(d_rirs, offs, lens, M, d_x, out_len, snr_db=snr, z=d_z, use_mfma=mfma)
    torch.cuda.synchronize()
    return y.cpu().numpy().astype(np.float64)


def _oracle(rirs, offs, lens, x, out_len, r, snr=None, z=None):
    L = int(lens[r])
    h = rirs[offs[r]:offs[r] + 8 * L].reshape(8, L).astype(np.float64)
    zz = None if z is None else z[r].astype(np.float64)
    return oracle.conv_room(h, x[r].astype(np.float64), out_len, snr_db=None if snr is None else float(snr[r]), z=zz)


def _check(got, ref, mfma):
    if mfma:
        rms = np.sqrt(np.mean((got - ref) ** 2)) / np.sqrt(np.mean(ref ** 2))
        assert rms <= TOL_BF16_RMS, rms
        return rms
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    assert err <= TOL_FP32, err
    return err


@pytest.mark.parametrize("mfma", [True, False])
def test_conv_ragged_small(H, mfma):
    lens = np.array([1, 37, 500, 1337, 2049])
    rirs, offs = scenes.synthetic_rirs(lens, 8, seed=3)
    rng = np.random.default_rng(4)
    x = rng.standard_normal((len(lens), 2000)).astype(np.float32)
    out_len = 1500
    got = _run(H, rirs, offs, lens, x, out_len, mfma=mfma)
    for r in range(len(lens)):
        ref = _oracle(rirs, offs, lens, x, out_len, r)
        e = _check(got[r], ref, mfma)
        sys.stdout.write(f"room {r} len {lens[r]} mfma={mfma} err {e:.3e}\n")


@pytest.mark.parametrize("mfma", [True, False])
def test_conv_noise_hits_snr(H, mfma):
    lens = np.array([300, 800])
    rirs, offs = scenes.synthetic_rirs(lens, 8, seed=5)
    rng = np.random.default_rng(6)
    x = rng.standard_normal((2, 3000)).astype(np.float32)
    out_len = 2500
    snr = np.array([3.0, 27.5], dtype=np.float32)
    z = rng.standard_normal((2, 8, out_len)).astype(np.float32)
    got = _run(H, rirs, offs, lens, x, out_len, snr=snr, z=z, mfma=mfma)
    for r in range(2):
        ref = _oracle(rirs, offs, lens, x, out_len, r, snr=snr, z=z)
        _check(got[r], ref, mfma)


def test_conv_full_size_sampled(H):
    # 256 rooms with the RIR lengths of the c4 workload, 1 s sources; 4 rooms checked in full
    b = scenes.c4()
    lens = b["rir_len"]
    rirs, offs = scenes.synthetic_rirs(lens, 8, seed=8)
    got = _run(H, rirs, offs, lens, b["x"], 16000, snr=b["snr_db"], z=b["z"], mfma=True)
    assert np.all(np.isfinite(got))
    for r in [0, 77, 190, 255]:
        ref = _oracle(rirs, offs, lens, b["x"], 16000, r, snr=b["snr_db"], z=b["z"])
        rms = _check(got[r], ref, True)
        sys.stdout.write(f"c4 room {r} len {lens[r]} rel rms {rms:.3e}\n")


def test_conv_argument_errors(H):
    import torch
    d = torch.zeros(16, device="cuda")
    with pytest.raises(ism.IsmError):
        H.convolve_batch(d, [0], [0], 8, torch.zeros((1, 4), device="cuda"), 4)
    with pytest.raises(ism.IsmError):   # MFMA path takes 8 microphones
        H.convolve_batch(d, [0], [2], 2, torch.zeros((1, 4), device="cuda"), 4, use_mfma=True)


def test_caller_outputs_are_checked(H):
    # a caller-supplied output that is too small, of another type or not contiguous is
    # refused before any launch
    import torch
    L, beta, src, mic = [5.0, 4.0, 3.0], [0.9] * 6, [1.0, 1.2, 1.1], [[3.0, 2.5, 1.6]]
    with pytest.raises(ValueError):
        H.rir(L, beta, src, mic, 16000.0, 343.0, 2, 512, 81, out=torch.empty(511, device="cuda"))
    with pytest.raises(ValueError):
        H.rir(L, beta, src, mic, 16000.0, 343.0, 2, 512, 81, out=torch.empty(512, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        H.rir(L, beta, src, mic, 16000.0, 343.0, 2, 512, 81, out=torch.empty((512, 2), device="cuda")[:, 0])
    d = torch.zeros(16, device="cuda")
    with pytest.raises(ValueError):
        H.convolve_batch(d, [0], [4], 1, torch.zeros((1, 4), device="cuda"), 4, use_mfma=False,
                         out=torch.empty(3, device="cuda"))
    with pytest.raises(ValueError):     # rirs shorter than offset + M x rir_len
        H.convolve_batch(d, [0], [9], 2, torch.zeros((1, 4), device="cuda"), 4, use_mfma=False)
    with pytest.raises(ValueError):     # source of another type
        H.convolve_batch(d, [0], [4], 1, torch.zeros((1, 4), dtype=torch.float64, device="cuda"), 4, use_mfma=False)
    with pytest.raises(ValueError):
        H.rir_t30(torch.ones(64, dtype=torch.float64, device="cuda"), 16000.0)
    out = H.rir(L, beta, src, mic, 16000.0, 343.0, 2, 512, 81, out=torch.empty(512, device="cuda"))
    torch.cuda.synchronize()
    assert torch.isfinite(out).all() and out.abs().max() > 0
